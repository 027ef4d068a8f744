"""FP64 CPU oracle of the Lévy LIBOR Monte Carlo path.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP implementation in ``paper_1006_3340_amd`` and imports nothing
from it; both are driven by the input generators in ``workloads``.

Layout: ``rule.py`` builds the 64-node quadrature rule over the NIG Lévy
measure (numpy Gauss-Legendre + scipy Bessel K_1); ``lll_oracle.c`` runs the
Euler paths, the drift of eq. (LIBOR-drift-PT) by its literal product form,
and the caplet payoff sums of eq. (caplet); this module marshals arguments
and forms prices from path sums.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

from . import rule

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lll_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblll_oracle.so")

FULL, PICARD, FROZEN, FIRST_ORDER, SECOND_ORDER = 0, 1, 2, 3, 4
NIG, BROWNIAN = 0, 1


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-std=c11", "-D_GNU_SOURCE", "-O2", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Model(ctypes.Structure):
    _fields_ = [
        ("n_rates", ctypes.c_int32),
        ("steps_per_period", ctypes.c_int32),
        ("n_strikes", ctypes.c_int32),
        ("driver", ctypes.c_int32),
        ("n_nodes", ctypes.c_int32),
        ("stream_word", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("product", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("tenor", ctypes.POINTER(ctypes.c_double)),
        ("delta", ctypes.POINTER(ctypes.c_double)),
        ("L0", ctypes.POINTER(ctypes.c_double)),
        ("vol", ctypes.POINTER(ctypes.c_double)),
        ("strikes", ctypes.POINTER(ctypes.c_double)),
        ("x", ctypes.POINTER(ctypes.c_double)),
        ("w", ctypes.POINTER(ctypes.c_double)),
        ("alpha", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("delta_nig", ctypes.c_double),
        ("c", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_create.restype = ctypes.c_void_p
        lib.oracle_create.argtypes = [ctypes.POINTER(_Model)]
        lib.oracle_destroy.argtypes = [ctypes.c_void_p]
        for fn in ("oracle_kappa_table", "oracle_E_table", "oracle_b0_table", "oracle_dt_table"):
            getattr(lib, fn).restype = dp
            getattr(lib, fn).argtypes = [ctypes.c_void_p]
        lib.oracle_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32),
                                             ctypes.POINTER(ctypes.c_uint32),
                                             ctypes.POINTER(ctypes.c_uint32)]
        lib.oracle_uniform.restype = ctypes.c_double
        lib.oracle_uniform.argtypes = [ctypes.c_uint32]
        lib.oracle_increment.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, dp, dp,
                                         ctypes.POINTER(ctypes.c_uint32)]
        lib.oracle_drift.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, dp, dp]
        lib.oracle_drift_first_order.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, dp, dp]
        lib.oracle_drift_second_order.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, dp, dp]
        lib.oracle_paths.argtypes = [ctypes.c_void_p, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, dp, dp]
        lib.oracle_paths.restype = ctypes.c_int
        lib.oracle_price_sums.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_int, dp, dp, dp, dp, dp]
        lib.oracle_increments.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                                          ctypes.c_int64, dp, dp]
        lib.oracle_price_sums.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def philox4x32_10(ctr, key) -> np.ndarray:
    """Raw Philox-4x32-10 words for one 128-bit counter and 64-bit key."""
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib.oracle_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def uniform(word: int) -> float:
    return _load().oracle_uniform(ctypes.c_uint32(int(word) & 0xFFFFFFFF))


class Oracle:
    """FP64 oracle bound to one term structure (see ``workloads.TermStructure``)."""

    def __init__(self, ts, seed: int = 1, tag: int = 0, nodes=None):
        lib = _load()
        ts.validate_shapes()
        self.ts = ts
        self.seed = int(seed)
        self.N = ts.n_rates
        self.S = ts.n_strikes
        self.s = ts.steps_per_period
        self.K = self.N * self.s
        f64 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float64))
        self._tenor = f64(ts.tenor)
        self._delta = f64(ts.delta)
        self._L0 = f64(ts.L0)
        self._vol = f64(ts.vol)
        self._strikes = f64(ts.strikes)
        if ts.driver == NIG:
            if nodes is None:
                x, W, info = rule.quadrature_rule(ts.alpha, ts.beta, ts.delta_nig, ts.vol,
                                                  ts.tenor, ts.steps_per_period)
                self.rule_info = info
            else:
                x, W = nodes
                self.rule_info = None
            self.x = f64(x)
            self.W = f64(W)
        else:
            self.x = np.zeros(1)
            self.W = np.zeros(1)
            self.rule_info = None
        m = _Model()
        m.n_rates = self.N
        m.steps_per_period = self.s
        m.n_strikes = self.S
        m.driver = int(ts.driver)
        m.n_nodes = len(self.x) if ts.driver == NIG else 0
        m.stream_word = (int(ts.struct_id) & 0xFFFFFF) | ((int(tag) & 0xFF) << 24)
        m.seed = self.seed
        m.product = int(getattr(ts, "product", 0))
        m.tenor, m.delta, m.L0 = _dp(self._tenor), _dp(self._delta), _dp(self._L0)
        m.vol, m.strikes = _dp(self._vol), _dp(self._strikes)
        m.x, m.w = _dp(self.x), _dp(self.W)
        m.alpha, m.beta, m.delta_nig, m.c = ts.alpha, ts.beta, ts.delta_nig, ts.c
        self._model = m
        self._ctx = lib.oracle_create(ctypes.byref(m))
        if not self._ctx:
            raise MemoryError("oracle_create failed")
        self._lib = lib
        Q = m.n_nodes
        self.kappa = np.ctypeslib.as_array(lib.oracle_kappa_table(self._ctx),
                                           shape=(self.K, self.N)).copy()
        self.b0 = np.ctypeslib.as_array(lib.oracle_b0_table(self._ctx),
                                        shape=(self.K, self.N)).copy()
        self.dt = np.ctypeslib.as_array(lib.oracle_dt_table(self._ctx), shape=(self.K,)).copy()
        if Q > 0:
            self.E = np.ctypeslib.as_array(lib.oracle_E_table(self._ctx),
                                           shape=(self.K, self.N, Q)).copy()
        else:
            self.E = None

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx:
            self._lib.oracle_destroy(ctx)
            self._ctx = None

    # -- pieces --------------------------------------------------------------
    def increment(self, k: int, p: int):
        """(V, dH, words) for step k of path p."""
        V = ctypes.c_double()
        dH = ctypes.c_double()
        w = (ctypes.c_uint32 * 4)()
        self._lib.oracle_increment(self._ctx, int(k), int(p), ctypes.byref(V),
                                   ctypes.byref(dH), w)
        return V.value, dH.value, np.array(list(w), dtype=np.uint32)

    def increments(self, k: int, p0: int, n: int):
        """(V, dH) arrays of step k for paths p0 .. p0+n-1."""
        V = np.zeros(n)
        dH = np.zeros(n)
        self._lib.oracle_increments(self._ctx, int(k), int(p0), int(n), _dp(V), _dp(dH))
        return V, dH

    def drift(self, k: int, L: np.ndarray, order: int = 0) -> np.ndarray:
        """Drift b(t_k, T_i) of the live rates at step k for given rates L (len N);
        order 1 / 2: its expansion of eq. (drifta) / (drifta2) instead."""
        L = np.ascontiguousarray(np.asarray(L, dtype=np.float64))
        b = np.zeros(self.N)
        first = k // self.s
        fn = {0: self._lib.oracle_drift, 1: self._lib.oracle_drift_first_order,
              2: self._lib.oracle_drift_second_order}[order]
        fn(self._ctx, int(k), int(first), _dp(L), _dp(b))
        b[:first] = np.nan
        return b

    def paths(self, scheme: int, path_indices) -> tuple:
        """Per-path fixings (Lfix, Dfix), each [n, N]."""
        idx = np.ascontiguousarray(np.asarray(path_indices, dtype=np.int64))
        n = len(idx)
        Lf = np.zeros((n, self.N))
        Df = np.zeros((n, self.N))
        self._lib.oracle_paths(self._ctx, int(scheme),
                               idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n,
                               _dp(Lf), _dp(Df))
        return Lf, Df

    def price_sums(self, scheme: int, n_paths: int, path0: int = 0, threads: int = 0) -> dict:
        N, S = self.N, self.S
        sp = np.zeros((N, S)); sp2 = np.zeros((N, S)); itm = np.zeros((N, S))
        mart = np.zeros(N)
        mart2 = np.zeros(N)
        used = self._lib.oracle_price_sums(self._ctx, int(scheme), int(path0), int(n_paths),
                                           int(threads), _dp(sp), _dp(sp2), _dp(itm), _dp(mart),
                                           _dp(mart2))
        if used < 0:
            raise MemoryError("oracle_price_sums failed")
        return {"sum_p": sp, "sum_p2": sp2, "n_itm": itm, "sum_mart": mart,
                "sum_mart2": mart2, "n_paths": int(n_paths), "threads": int(used)}

    # -- prices --------------------------------------------------------------
    def B0_Tstar(self) -> float:
        """B(0, T_*) = B(0, T_1) / prod_{l=1}^{N} (1 + delta_l L(0, T_l))."""
        return float(self.ts.B0_T1 / np.prod(1.0 + self._delta * self._L0))

    def price(self, scheme: int, n_paths: int, path0: int = 0, threads: int = 0) -> dict:
        """Caplet prices, standard errors and martingale residuals (eq. (caplet))."""
        sums = self.price_sums(scheme, n_paths, path0, threads)
        return finish(sums, self._delta, self._L0, self.B0_Tstar(),
                      swaptions=int(getattr(self.ts, "product", 0)) == 1)


def finish(sums: dict, delta: np.ndarray, L0: np.ndarray, B0_Tstar: float,
           swaptions: bool = False) -> dict:
    """Prices delta_i B(0,T_*) mean(payoff) (swaptions: B(0,T_*) mean(payoff)),
    standard errors and martingale residuals
    mean(prod_{l>=i}(1 + delta_l L_l)) - prod_{l>=i}(1 + delta_l L(0,T_l))."""
    n = sums["n_paths"]
    scale = (np.ones_like(delta) if swaptions else delta)[:, None] * B0_Tstar
    mean = sums["sum_p"] / n
    var = np.maximum(sums["sum_p2"] / n - mean * mean, 0.0)
    se = scale * np.sqrt(var / max(n - 1, 1))
    fwd = np.array([np.prod(1.0 + delta[i:] * L0[i:]) for i in range(len(L0))])
    mm = sums["sum_mart"] / n
    mvar = np.maximum(sums["sum_mart2"] / n - mm * mm, 0.0)
    return {"price": scale * mean, "stderr": se,
            "mart_resid": mm - fwd, "mart_se": np.sqrt(mvar / max(n - 1, 1)),
            "n_itm": sums["n_itm"], **{k: v for k, v in sums.items() if k != "n_itm"}}
