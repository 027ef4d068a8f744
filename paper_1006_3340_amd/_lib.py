"""ctypes binding of the C ABI in include/lll.h (argument marshalling only).

Every step of the computation runs in the HIP library ``liblll.so``; this
module converts numpy inputs to the ABI's plain pointers and sizes, turns
status codes into exceptions and returns numpy outputs.  There is no
fallback: if the library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblll.so")

LLL_OK = 0
STATUS = {0: "LLL_OK", -1: "LLL_EINVAL", -2: "LLL_EMOMENT", -3: "LLL_ENOMEM", -4: "LLL_EHIP",
          -5: "LLL_EUNSUPPORTED", -6: "LLL_ENUMERIC"}
FULL, PICARD, FROZEN, FIRST_ORDER, SECOND_ORDER, PICARD_MP, EXACT, MLP_DRIFT = 0, 1, 2, 3, 4, 5, 6, 7
CAPLETS, SWAPTIONS = 0, 1
FP32, FP64 = 0, 1
N_MAX, N_MAX_MP, N_MAX_FP64, N_MAX_EXACT, S_MAX, Q = 40, 64, 24, 20, 8, 64

EXPORTS = ["lll_version", "lll_last_error", "lll_plan_create", "lll_plan_execute",
           "lll_plan_results", "lll_plan_sums", "lll_plan_partials", "lll_plan_destroy",
           "lll_price_caplets", "lll_philox", "lll_sampler_math", "lll_plan_increments",
           "lll_plan_tables",
           "lll_plan_drift", "lll_plan_set_timing", "lll_plan_timing", "lll_batch_create",
           "lll_batch_execute", "lll_batch_results", "lll_batch_set_timing", "lll_batch_timing",
           "lll_batch_destroy", "lll_plan_greeks", "lll_plan_greeks_results", "lll_plan_greeks_vjp",
           "lll_plan_greeks_vjp_results", "lll_caplet_greeks", "lll_price_caplets_batched",
           "lll_fp32_fma_peak", "lll_fp32_mix_peak", "lll_fp32_mfma_peak", "lll_price_caplets_static",
           "lll_mlp_create", "lll_mlp_destroy", "lll_mlp_params", "lll_mlp_generate",
           "lll_mlp_info", "lll_mlp_set_box", "lll_mlp_pairs", "lll_mlp_train", "lll_mlp_eval",
           "lll_plan_execute_mlp", "lll_plan_mlp_stats", "lll_mlp_train_dev",
           "lll_mlp_optimizer_state", "lll_mlp_copy_pairs_dev", "lll_plan_set_inputs_dev",
           "lll_plan_results_dev", "lll_plan_attach_mlp", "lll_plan_greeks_vjp_dev",
           "lll_plan_greeks_vjp_results_dev", "lll_plan_greeks_results_dev"]
MLP_PARAMS, MLP_INPUTS = 14593, 96


class LLLError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS.get(code, code)}: {message}")
        self.code = code


class TermStructureC(ctypes.Structure):
    _fields_ = [
        ("n_rates", ctypes.c_int32),
        ("steps_per_period", ctypes.c_int32),
        ("n_strikes", ctypes.c_int32),
        ("driver", ctypes.c_int32),
        ("struct_id", ctypes.c_uint32),
        ("product", ctypes.c_int32),
        ("tenor", ctypes.POINTER(ctypes.c_double)),
        ("delta", ctypes.POINTER(ctypes.c_double)),
        ("L0", ctypes.POINTER(ctypes.c_double)),
        ("B0_T1", ctypes.c_double),
        ("vol", ctypes.POINTER(ctypes.c_double)),
        ("strikes", ctypes.POINTER(ctypes.c_double)),
        ("alpha", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("delta_nig", ctypes.c_double),
        ("c", ctypes.c_double),
    ]


_lib = None


def load():
    """Load liblll.so (built by ``__graft_entry__.build()``); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, u64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.lll_version.restype = ctypes.c_char_p
    lib.lll_last_error.restype = ctypes.c_char_p
    lib.lll_plan_create.argtypes = [ctypes.POINTER(TermStructureC), i32, i64, ctypes.POINTER(vp)]
    lib.lll_plan_execute.argtypes = [vp, i32, i64, i64, u64, vp, vp]
    lib.lll_plan_results.argtypes = [vp, dp, dp, dp, dp, dp, vp]
    lib.lll_plan_sums.argtypes = [vp, dp, vp]
    lib.lll_plan_partials.argtypes = [vp, dp, i64, vp]
    lib.lll_plan_destroy.argtypes = [vp]
    lib.lll_price_caplets.argtypes = [ctypes.POINTER(TermStructureC), i64, i32, u64, i32, dp, dp,
                                      dp, vp]
    lib.lll_price_caplets_static.argtypes = lib.lll_price_caplets.argtypes
    dpp = ctypes.POINTER(dp)
    lib.lll_price_caplets_batched.argtypes = [ctypes.POINTER(TermStructureC), i32, i64, i32, u64,
                                              dpp, dpp, vp]
    lib.lll_fp32_fma_peak.argtypes = [dp, vp]
    lib.lll_fp32_mix_peak.argtypes = [dp, vp]
    lib.lll_fp32_mfma_peak.argtypes = [dp, vp]
    lib.lll_philox.argtypes = [u32p, u32p, i64, u32p, vp]
    lib.lll_sampler_math.argtypes = [ctypes.c_int, dp, i64, dp, vp]
    lib.lll_plan_increments.argtypes = [vp, i32, i64, i64, u64, dp, dp, vp]
    lib.lll_plan_tables.argtypes = [vp, dp, dp, dp, dp, dp, vp]
    lib.lll_plan_drift.argtypes = [vp, i32, dp, i64, dp, vp]
    fp = ctypes.POINTER(ctypes.c_float)
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int)
    lib.lll_mlp_create.argtypes = [u64, ctypes.POINTER(vp)]
    lib.lll_mlp_destroy.argtypes = [vp]
    lib.lll_mlp_params.argtypes = [vp, fp, fp]
    lib.lll_mlp_generate.argtypes = [vp, vp, i64, i32, u64, i64p, vp]
    lib.lll_mlp_info.argtypes = [vp, fp, i64p]
    lib.lll_mlp_set_box.argtypes = [vp, fp]
    lib.lll_mlp_pairs.argtypes = [vp, i64p, i64, fp, i32p, i32p, fp, fp]
    lib.lll_mlp_train.argtypes = [vp, i32, i32, ctypes.c_float, u64, fp, vp]
    lib.lll_mlp_eval.argtypes = [vp, fp, fp, i64, fp, fp, fp, vp]
    lib.lll_mlp_train_dev.argtypes = [vp, vp, vp, i64, ctypes.c_float, i32, i32, ctypes.c_float,
                                      u64, vp, vp]
    lib.lll_mlp_optimizer_state.argtypes = [vp, fp, fp, i64p]
    lib.lll_mlp_copy_pairs_dev.argtypes = [vp, vp, vp, i64, vp]
    lib.lll_plan_execute_mlp.argtypes = [vp, vp, i32, i64, u64, i32, vp, vp]
    lib.lll_plan_mlp_stats.argtypes = [vp, dp, vp]
    lib.lll_plan_greeks.argtypes = [vp, i64, u64, vp]
    lib.lll_plan_greeks_results.argtypes = [vp, dp, dp, dp, vp]
    lib.lll_plan_greeks_vjp.argtypes = [vp, i64, u64, dp, vp]
    lib.lll_plan_greeks_vjp_results.argtypes = [vp, dp, dp, dp, vp]
    lib.lll_caplet_greeks.argtypes = [ctypes.POINTER(TermStructureC), i64, u64, dp, dp, dp, vp]
    lib.lll_batch_create.argtypes = [ctypes.POINTER(TermStructureC), i32, i64, ctypes.POINTER(vp)]
    lib.lll_batch_execute.argtypes = [vp, i32, i64, u64, vp]
    lib.lll_batch_results.argtypes = [vp, i32, dp, dp, dp, dp, dp, vp]
    lib.lll_batch_set_timing.argtypes = [vp, i32]
    lib.lll_batch_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_float)]
    lib.lll_batch_destroy.argtypes = [vp]
    lib.lll_plan_set_inputs_dev.argtypes = [vp, vp, vp, vp]
    lib.lll_plan_results_dev.argtypes = [vp, vp, vp, vp, vp]
    lib.lll_plan_attach_mlp.argtypes = [vp, vp]
    lib.lll_plan_greeks_vjp_dev.argtypes = [vp, i64, u64, vp, vp]
    lib.lll_plan_greeks_vjp_results_dev.argtypes = [vp, vp, vp, vp, vp]
    lib.lll_plan_greeks_results_dev.argtypes = [vp, vp, vp, vp, vp]
    lib.lll_plan_set_timing.argtypes = [vp, i32]
    lib.lll_plan_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_float)]
    for name in EXPORTS:
        if name not in ("lll_version", "lll_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != LLL_OK:
        msg = load().lll_last_error().decode(errors="replace")
        raise LLLError(rc, msg)


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def stream_handle(stream) -> Optional[int]:
    """hipStream_t of a torch stream (or an int handle); None = default stream."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def dev_f64(t, n: int, name: str) -> Optional[int]:
    """Address of a contiguous float64 device tensor with at least n elements
    (None passes NULL); anything else raises before the library is called."""
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous() and t.numel() >= n):
        raise ValueError(f"{name}: needs a contiguous float64 CUDA tensor of >= {n} elements")
    return int(t.data_ptr())


def device_ptr(t) -> Optional[int]:
    """Device address of a torch tensor (or an int address); None passes NULL."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return int(t.data_ptr())


class _TS:
    """Keeps the numpy arrays behind one lll_term_structure alive."""

    def __init__(self, ts):
        ts.validate_shapes()
        f64 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float64))
        self.arrays = [f64(ts.tenor), f64(ts.delta), f64(ts.L0), f64(ts.vol), f64(ts.strikes)]
        c = TermStructureC()
        c.n_rates = ts.n_rates
        c.steps_per_period = ts.steps_per_period
        c.n_strikes = ts.n_strikes
        c.driver = int(ts.driver)
        c.struct_id = int(ts.struct_id) & 0xFFFFFFFF
        c.product = int(getattr(ts, "product", 0))
        c.tenor, c.delta, c.L0, c.vol, c.strikes = [_dp(a) for a in self.arrays]
        c.B0_T1 = float(ts.B0_T1)
        c.alpha, c.beta, c.delta_nig, c.c = (float(ts.alpha), float(ts.beta),
                                             float(ts.delta_nig), float(ts.c))
        self.c = c


class Plan:
    """lll_plan: one term structure resident on the current HIP device."""

    def __init__(self, ts, precision: int = FP32, max_paths: int = 1 << 20):
        self.lib = load()
        self._ts = _TS(ts)
        self.N, self.S = ts.n_rates, ts.n_strikes
        self.K = ts.n_rates * ts.steps_per_period
        self.max_paths = int(max_paths)
        h = ctypes.c_void_p()
        _check(self.lib.lll_plan_create(ctypes.byref(self._ts.c), int(precision),
                                        int(max_paths), ctypes.byref(h)))
        self.h = h
        self.n_paths = 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.lll_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def execute(self, scheme: int, n_paths: int, seed: int = 1, path_offset: int = 0,
                path_fix=None, stream=None):
        _check(self.lib.lll_plan_execute(self.h, int(scheme), int(n_paths), int(path_offset),
                                         int(seed), device_ptr(path_fix), stream_handle(stream)))
        self.n_paths = int(n_paths)

    def set_timing(self, enable: bool = True):
        _check(self.lib.lll_plan_set_timing(self.h, 1 if enable else 0))

    def set_inputs_dev(self, L0=None, vol_shift=None, stream=None):
        """lll_plan_set_inputs_dev: forwards L0 [N] and per-rate vol shifts [N]
        from float64 device tensors (either may be None), asynchronous."""
        _check(self.lib.lll_plan_set_inputs_dev(self.h, dev_f64(L0, self.N, "L0"),
                                                dev_f64(vol_shift, self.N, "vol_shift"),
                                                stream_handle(stream)))

    def results_dev(self, price=None, stderr=None, mart_resid=None, stream=None):
        """lll_plan_results_dev: the last execute's prices [N][S], standard
        errors [N][S] and martingale residuals [N] into float64 device tensors."""
        NS = self.N * self.S
        _check(self.lib.lll_plan_results_dev(self.h, dev_f64(price, NS, "price"),
                                             dev_f64(stderr, NS, "stderr"),
                                             dev_f64(mart_resid, self.N, "mart_resid"),
                                             stream_handle(stream)))

    def attach_mlp(self, mlp):
        """lll_plan_attach_mlp: the network scheme MLP_DRIFT uses (None detaches)."""
        _check(self.lib.lll_plan_attach_mlp(self.h, mlp.h if mlp is not None else None))
        self._mlp = mlp   # the network must outlive its use by the plan

    def greeks_vjp_dev(self, n_paths: int, weights, seed: int = 1, stream=None):
        """lll_plan_greeks_vjp_dev: weights [N] from a float64 device tensor."""
        _check(self.lib.lll_plan_greeks_vjp_dev(self.h, int(n_paths), int(seed),
                                                dev_f64(weights, self.N, "weights"),
                                                stream_handle(stream)))
        self.n_paths = int(n_paths)

    def greeks_vjp_results_dev(self, price=None, vjp_L0=None, vjp_vol=None, stream=None):
        N = self.N
        _check(self.lib.lll_plan_greeks_vjp_results_dev(
            self.h, dev_f64(price, N, "price"), dev_f64(vjp_L0, N, "vjp_L0"),
            dev_f64(vjp_vol, N, "vjp_vol"), stream_handle(stream)))

    def greeks_results_dev(self, price=None, dP_dL0=None, dP_dvol=None, stream=None):
        N = self.N
        _check(self.lib.lll_plan_greeks_results_dev(
            self.h, dev_f64(price, N, "price"), dev_f64(dP_dL0, N * N, "dP_dL0"),
            dev_f64(dP_dvol, N * N, "dP_dvol"), stream_handle(stream)))

    def timing(self) -> dict:
        """Durations (ms) of the last timed execute's stages, from HIP events."""
        ms = (ctypes.c_float * 3)()
        _check(self.lib.lll_plan_timing(self.h, ms))
        return {"precompute": ms[0], "paths": ms[1], "reduce": ms[2]}

    def execute_mlp(self, mlp, use_net: bool, n_paths: int, seed: int = 1, judge_stride: int = 0,
                    path_fix=None, stream=None):
        """Pricing pass with the surrogate drift (use_net) or the first-order expansion alone."""
        _check(self.lib.lll_plan_execute_mlp(self.h, mlp.h if mlp is not None else None,
                                             1 if use_net else 0, int(n_paths), int(seed),
                                             int(judge_stride), device_ptr(path_fix),
                                             stream_handle(stream)))
        self.n_paths = int(n_paths)

    def mlp_stats(self, stream=None) -> dict:
        out = np.zeros(8)
        _check(self.lib.lll_plan_mlp_stats(self.h, _dp(out), stream_handle(stream)))
        return {"rate_steps": out[0], "fallbacks": out[1], "judged": out[2],
                "judge_abs_err": out[3], "judge_abs_quad": out[4], "judge_max_rel": out[5]}

    def greeks(self, n_paths: int, seed: int = 1, stream=None):
        """Enqueue the FULL pricing pass with the pathwise adjoint (lll_plan_greeks)."""
        _check(self.lib.lll_plan_greeks(self.h, int(n_paths), int(seed), stream_handle(stream)))
        self.n_paths = int(n_paths)

    def greeks_vjp(self, n_paths: int, weights, seed: int = 1, stream=None):
        """Enqueue the single-sweep vector-Jacobian product (lll_plan_greeks_vjp)."""
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(self.N))
        _check(self.lib.lll_plan_greeks_vjp(self.h, int(n_paths), int(seed), _dp(w),
                                            stream_handle(stream)))
        self.n_paths = int(n_paths)

    def greeks_vjp_results(self, stream=None) -> dict:
        N = self.N
        price = np.zeros(N); gL = np.zeros(N); gV = np.zeros(N)
        _check(self.lib.lll_plan_greeks_vjp_results(self.h, _dp(price), _dp(gL), _dp(gV),
                                                    stream_handle(stream)))
        return {"price": price, "vjp_L0": gL, "vjp_vol": gV}

    def greeks_results(self, stream=None) -> dict:
        N = self.N
        price = np.zeros(N); dL = np.zeros((N, N)); dV = np.zeros((N, N))
        _check(self.lib.lll_plan_greeks_results(self.h, _dp(price), _dp(dL), _dp(dV),
                                                stream_handle(stream)))
        return {"price": price, "dP_dL0": dL, "dP_dvol": dV}

    def results(self, stream=None) -> dict:
        N, S = self.N, self.S
        price = np.zeros((N, S)); se = np.zeros((N, S)); itm = np.zeros((N, S))
        mart = np.zeros(N); mse = np.zeros(N)
        _check(self.lib.lll_plan_results(self.h, _dp(price), _dp(se), _dp(mart), _dp(mse),
                                         _dp(itm), stream_handle(stream)))
        return {"price": price, "stderr": se, "mart_resid": mart, "mart_se": mse,
                "n_itm": itm, "n_paths": self.n_paths}

    def sums(self, stream=None) -> np.ndarray:
        out = np.zeros((self.N, 3 * self.S + 2))
        _check(self.lib.lll_plan_sums(self.h, _dp(out), stream_handle(stream)))
        return out

    def partials(self, stream=None) -> np.ndarray:
        waves = (self.n_paths + 63) // 64
        out = np.zeros((waves, self.N, 3 * self.S + 2))
        _check(self.lib.lll_plan_partials(self.h, _dp(out), out.size, stream_handle(stream)))
        return out

    def increments(self, k: int, p0: int, n: int, seed: int = 1, stream=None):
        V = np.zeros(n); dH = np.zeros(n)
        _check(self.lib.lll_plan_increments(self.h, int(k), int(p0), int(n), int(seed), _dp(V),
                                            _dp(dH), stream_handle(stream)))
        return V, dH

    def tables(self, stream=None) -> dict:
        K, N = self.K, self.N
        x = np.zeros(Q); w = np.zeros(Q); kap = np.zeros((K, N)); E = np.zeros((K, N, Q))
        b0 = np.zeros((K, N))
        _check(self.lib.lll_plan_tables(self.h, _dp(x), _dp(w), _dp(kap), _dp(E), _dp(b0),
                                        stream_handle(stream)))
        return {"x": x, "w": w, "kappa": kap, "E": E, "b0": b0}

    def drift(self, k: int, L: np.ndarray, stream=None) -> np.ndarray:
        L = np.ascontiguousarray(np.atleast_2d(np.asarray(L, dtype=np.float64)))
        b = np.zeros_like(L)
        _check(self.lib.lll_plan_drift(self.h, int(k), _dp(L), L.shape[0], _dp(b),
                                       stream_handle(stream)))
        return b


class Batch:
    """lll_batch: many term structures priced in one persistent launch (FP32)."""

    def __init__(self, structures, max_paths_each: int = 1 << 18):
        self.lib = load()
        self._ts = [_TS(ts) for ts in structures]
        self.shapes = [(ts.n_rates, ts.n_strikes) for ts in structures]
        arr = (TermStructureC * len(self._ts))(*[t.c for t in self._ts])
        self._arr = arr
        h = ctypes.c_void_p()
        _check(self.lib.lll_batch_create(arr, len(self._ts), int(max_paths_each), ctypes.byref(h)))
        self.h = h
        self.n_paths_each = 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.lll_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def execute(self, scheme: int, n_paths_each: int, seed: int = 1, stream=None):
        _check(self.lib.lll_batch_execute(self.h, int(scheme), int(n_paths_each), int(seed),
                                          stream_handle(stream)))
        self.n_paths_each = int(n_paths_each)

    def set_timing(self, enable: bool = True):
        _check(self.lib.lll_batch_set_timing(self.h, 1 if enable else 0))

    def timing(self) -> float:
        ms = ctypes.c_float()
        _check(self.lib.lll_batch_timing(self.h, ctypes.byref(ms)))
        return ms.value

    def results(self, index: int, stream=None) -> dict:
        N, S = self.shapes[index]
        price = np.zeros((N, S)); se = np.zeros((N, S)); itm = np.zeros((N, S))
        mart = np.zeros(N); mse = np.zeros(N)
        _check(self.lib.lll_batch_results(self.h, int(index), _dp(price), _dp(se), _dp(mart),
                                          _dp(mse), _dp(itm), stream_handle(stream)))
        return {"price": price, "stderr": se, "mart_resid": mart, "mart_se": mse,
                "n_itm": itm, "n_paths": self.n_paths_each}


def price_caplets(ts, n_paths: int, scheme: int = FULL, seed: int = 1, precision: int = FP32,
                  stream=None) -> dict:
    """lll_price_caplets: prices, standard errors and martingale residuals."""
    lib = load()
    t = _TS(ts)
    N, S = ts.n_rates, ts.n_strikes
    price = np.zeros((N, S)); se = np.zeros((N, S)); mart = np.zeros(N)
    _check(lib.lll_price_caplets(ctypes.byref(t.c), int(n_paths), int(scheme), int(seed),
                                 int(precision), _dp(price), _dp(se), _dp(mart),
                                 stream_handle(stream)))
    return {"price": price, "stderr": se, "mart_resid": mart}


def price_caplets_static(ts, n_paths: int, scheme: int = FULL, seed: int = 1,
                         precision: int = FP32, stream=None) -> dict:
    """lll_price_caplets_static: lll_price_caplets with every device buffer in
    the library's static workspace (no device allocation)."""
    lib = load()
    t = _TS(ts)
    N, S = ts.n_rates, ts.n_strikes
    price = np.zeros((N, S)); se = np.zeros((N, S)); mart = np.zeros(N)
    _check(lib.lll_price_caplets_static(ctypes.byref(t.c), int(n_paths), int(scheme), int(seed),
                                        int(precision), _dp(price), _dp(se), _dp(mart),
                                        stream_handle(stream)))
    return {"price": price, "stderr": se, "mart_resid": mart}


def fp32_fma_peak(stream=None) -> float:
    """lll_fp32_fma_peak: measured non-packed FP32 FMA throughput, TFLOP/s."""
    lib = load()
    out = np.zeros(1)
    _check(lib.lll_fp32_fma_peak(_dp(out), stream_handle(stream)))
    return float(out[0])


def fp32_mix_peak(stream=None) -> float:
    """lll_fp32_mix_peak: measured throughput of the quadrature recursion's
    instruction mix, TFLOP/s."""
    lib = load()
    out = np.zeros(1)
    _check(lib.lll_fp32_mix_peak(_dp(out), stream_handle(stream)))
    return float(out[0])


def fp32_mfma_peak(stream=None) -> float:
    """lll_fp32_mfma_peak: measured throughput of independent FP32 16x16x4
    matrix-core instructions, TFLOP/s."""
    lib = load()
    out = np.zeros(1)
    _check(lib.lll_fp32_mfma_peak(_dp(out), stream_handle(stream)))
    return float(out[0])


def price_caplets_batched(structures, n_paths_each: int, scheme: int = FULL, seed: int = 1,
                          stream=None) -> list:
    """lll_price_caplets_batched: prices and standard errors of every structure
    from one persistent launch."""
    lib = load()
    ts_c = [_TS(ts) for ts in structures]
    arr = (TermStructureC * len(ts_c))(*[t.c for t in ts_c])
    out = [{"price": np.zeros((ts.n_rates, ts.n_strikes)), "stderr": np.zeros((ts.n_rates, ts.n_strikes))}
           for ts in structures]
    dp = ctypes.POINTER(ctypes.c_double)
    prices = (dp * len(out))(*[_dp(o["price"]) for o in out])
    ses = (dp * len(out))(*[_dp(o["stderr"]) for o in out])
    _check(lib.lll_price_caplets_batched(arr, len(ts_c), int(n_paths_each), int(scheme), int(seed),
                                         prices, ses, stream_handle(stream)))
    return out


def _fp(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Mlp:
    """lll_mlp: the drift surrogate (weights, training data, optimiser state)."""

    def __init__(self, seed: int = 1):
        self.lib = load()
        h = ctypes.c_void_p()
        _check(self.lib.lll_mlp_create(int(seed), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.lll_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def params(self) -> np.ndarray:
        out = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(self.lib.lll_mlp_params(self.h, _fp(out), None))
        return out

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
        assert p.shape == (MLP_PARAMS,)
        _check(self.lib.lll_mlp_params(self.h, None, _fp(p)))

    def generate(self, plan: "Plan", n_paths: int, records: int, seed: int = 1, stream=None) -> int:
        n = ctypes.c_int64()
        _check(self.lib.lll_mlp_generate(self.h, plan.h, int(n_paths), int(records), int(seed),
                                         ctypes.byref(n), stream_handle(stream)))
        return n.value

    def info(self) -> dict:
        out = np.zeros(81, dtype=np.float32)
        n = ctypes.c_int64()
        _check(self.lib.lll_mlp_info(self.h, _fp(out), ctypes.byref(n)))
        return {"lo": out[:40].copy(), "hi": out[40:80].copy(), "sigma": float(out[80]),
                "n_pairs": n.value}

    def set_box(self, lo: np.ndarray, hi: np.ndarray):
        box = np.ascontiguousarray(np.concatenate([np.asarray(lo, dtype=np.float32).ravel(),
                                                   np.asarray(hi, dtype=np.float32).ravel()]))
        assert box.shape == (80,)
        _check(self.lib.lll_mlp_set_box(self.h, _fp(box)))

    def pairs(self, idx) -> dict:
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
        n = len(idx)
        st = np.zeros((n, 40), dtype=np.float32)
        k = np.zeros(n, dtype=np.int32); r = np.zeros(n, dtype=np.int32)
        lab = np.zeros(n, dtype=np.float32); feat = np.zeros((n, MLP_INPUTS), dtype=np.float32)
        i32p = ctypes.POINTER(ctypes.c_int)
        _check(self.lib.lll_mlp_pairs(self.h, idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      n, _fp(st), k.ctypes.data_as(i32p), r.ctypes.data_as(i32p),
                                      _fp(lab), _fp(feat)))
        return {"state": st, "k": k, "rate": r, "label": lab, "feat": feat}

    def train(self, n_steps: int, batch: int = 16384, lr: float = 2e-3, seed: int = 1,
              stream=None) -> np.ndarray:
        loss = np.zeros(n_steps, dtype=np.float32)
        _check(self.lib.lll_mlp_train(self.h, int(n_steps), int(batch), ctypes.c_float(lr),
                                      int(seed), _fp(loss), stream_handle(stream)))
        return loss

    def train_dev(self, feat, labels, sigma: float, n_steps: int, batch: int = 16384,
                  lr: float = 2e-3, seed: int = 1, loss=None, stream=None):
        """lll_mlp_train_dev on device tensors: feat [n][96] bfloat16, labels [n]
        float32, loss [n_steps] float32 (optional); asynchronous on `stream`."""
        n = int(labels.shape[0])
        assert tuple(feat.shape) == (n, MLP_INPUTS) and feat.element_size() == 2
        assert labels.element_size() == 4
        assert feat.is_contiguous() and labels.is_contiguous()
        if loss is not None:
            assert loss.numel() >= n_steps and loss.element_size() == 4 and loss.is_contiguous()
        _check(self.lib.lll_mlp_train_dev(self.h, device_ptr(feat), device_ptr(labels), n,
                                          ctypes.c_float(sigma), int(n_steps), int(batch),
                                          ctypes.c_float(lr), int(seed), device_ptr(loss),
                                          stream_handle(stream)))

    def optimizer_state(self) -> dict:
        m = np.zeros(MLP_PARAMS, dtype=np.float32)
        v = np.zeros(MLP_PARAMS, dtype=np.float32)
        t = ctypes.c_int64()
        _check(self.lib.lll_mlp_optimizer_state(self.h, _fp(m), _fp(v), ctypes.byref(t)))
        return {"m": m, "v": v, "step": t.value}

    def copy_pairs_dev(self, feat, labels, stream=None):
        """lll_mlp_copy_pairs_dev into device tensors feat [>=n][96] (2-byte
        elements) and labels [>=n] float32."""
        assert feat.element_size() == 2 and labels.element_size() == 4
        assert feat.is_contiguous() and labels.is_contiguous() and feat.shape[-1] == MLP_INPUTS
        _check(self.lib.lll_mlp_copy_pairs_dev(self.h, device_ptr(feat), device_ptr(labels),
                                               min(int(feat.shape[0]), int(labels.shape[0])),
                                               stream_handle(stream)))

    def eval(self, feat: np.ndarray, target: Optional[np.ndarray] = None, stream=None) -> dict:
        feat = np.ascontiguousarray(np.asarray(feat, dtype=np.float32))
        n = feat.shape[0]
        y = np.zeros(n, dtype=np.float32)
        out = {"y": y}
        if target is not None:
            target = np.ascontiguousarray(np.asarray(target, dtype=np.float32))
            g = np.zeros(MLP_PARAMS, dtype=np.float32); loss = np.zeros(1, dtype=np.float32)
            _check(self.lib.lll_mlp_eval(self.h, _fp(feat), _fp(target), n, _fp(y), _fp(g),
                                         _fp(loss), stream_handle(stream)))
            out.update(grad=g, loss=float(loss[0]))
        else:
            _check(self.lib.lll_mlp_eval(self.h, _fp(feat), None, n, _fp(y), None, None,
                                         stream_handle(stream)))
        return out


def caplet_greeks(ts, n_paths: int, seed: int = 1, stream=None) -> dict:
    """lll_caplet_greeks: caplet prices (strike 0) and their pathwise derivatives
    with respect to L(0, T_l) and to parallel shifts of each rate's vol curve."""
    lib = load()
    t = _TS(ts)
    N = ts.n_rates
    price = np.zeros(N); dL = np.zeros((N, N)); dV = np.zeros((N, N))
    _check(lib.lll_caplet_greeks(ctypes.byref(t.c), int(n_paths), int(seed), _dp(price), _dp(dL),
                                 _dp(dV), stream_handle(stream)))
    return {"price": price, "dP_dL0": dL, "dP_dvol": dV}


def philox(ctr: np.ndarray, key: np.ndarray, stream=None) -> np.ndarray:
    """lll_philox: Philox-4x32-10 words computed on the device."""
    lib = load()
    ctr = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(-1, 4))
    key = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(-1, 2))
    n = ctr.shape[0]
    out = np.zeros((n, 4), dtype=np.uint32)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    _check(lib.lll_philox(ctr.ctypes.data_as(u32p), key.ctypes.data_as(u32p), n,
                          out.ctypes.data_as(u32p), stream_handle(stream)))
    return out


SAMPLER_ROUTINES = {"log": 0, "sinpi": 1, "cospi": 2, "sqrt": 3, "div": 4}


def sampler_math(routine: str, x: np.ndarray, stream=None) -> np.ndarray:
    """lll_sampler_math: one of the driver increment's FP64 routines ("log",
    "sinpi", "cospi", "sqrt"; "div" takes an (n, 2) array of a, b pairs)
    evaluated on the device."""
    lib = load()
    fn = SAMPLER_ROUTINES[routine]
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    n = x.shape[0]
    if fn == SAMPLER_ROUTINES["div"]:
        x = np.ascontiguousarray(x.reshape(-1, 2))
        n = x.shape[0]
    out = np.zeros(n, dtype=np.float64)
    _check(lib.lll_sampler_math(fn, _dp(x), n, _dp(out), stream_handle(stream)))
    return out


def version() -> str:
    return load().lll_version().decode()
