"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/lll.h declares, and rejects malformed inputs with the
documented status codes before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "lll.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lll_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_header_functions():
    import paper_1006_3340_amd._lib as L
    lib = L.load()
    names = header_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.EXPORTS)


def test_version_string():
    import paper_1006_3340_amd as lll
    assert "gfx950" in lll.version()


def _expect(code, ts, **kw):
    import paper_1006_3340_amd as lll
    with pytest.raises(lll.LLLError) as ei:
        lll.Plan(ts, **kw)
    assert ei.value.code == code, str(ei.value)
    return str(ei.value)


def test_validation_errors():
    EINVAL, EMOMENT, EUNSUP = -1, -2, -5
    ts = workloads.plain_fp64()
    _expect(EINVAL, ts.copy(L0=-ts.L0))
    L0 = ts.L0.copy(); L0[3] = np.nan
    _expect(EINVAL, ts.copy(L0=L0))
    tenor = ts.tenor.copy(); tenor[4] = tenor[3]
    _expect(EINVAL, ts.copy(tenor=tenor))
    delta = ts.delta.copy(); delta[2] = 0.3
    _expect(EINVAL, ts.copy(delta=delta))
    _expect(EINVAL, ts.copy(alpha=3.0, beta=-4.0))          # alpha <= |beta|
    _expect(EINVAL, ts.copy(delta_nig=0.0))
    _expect(EINVAL, ts.copy(steps_per_period=0, vol=ts.vol[:0]))
    vol = ts.vol.copy(); vol[5, 7] = np.inf
    _expect(EINVAL, ts.copy(vol=vol))
    _expect(EINVAL, ts.copy(driver=7))
    _expect(EINVAL, ts.copy(driver=1, c=-1.0))
    _expect(EINVAL, ts, max_paths=0)
    _expect(EINVAL, ts, precision=5)
    _expect(EINVAL, ts.copy(strikes=np.zeros((10, 9))))  # more than 8 strikes
    # drift integral diverges: the live vols sum beyond alpha - beta
    msg = _expect(EMOMENT, ts.copy(vol=ts.vol * 20.0))
    assert "Lambda" in msg
    # the paper's own example sits just inside the moment condition
    k = workloads.kluge_example()
    _expect(EMOMENT, k.copy(vol=k.vol * 1.05))
    # FP64 path kernel only up to 24 rates
    _expect(EUNSUP, workloads.learned_drift(), precision=1)
    big = workloads.make_structure(65, 0.25, 0.03, 2, lambda t, T, r: 0.1, [1.0])
    _expect(EINVAL, big)                                  # beyond LLL_N_MAX_MP
    bad = ts.copy()
    bad.product = 2                                       # neither caplets nor swaptions
    _expect(EINVAL, bad)


def test_inspection_entry_points_validate():
    import paper_1006_3340_amd as lll
    with pytest.raises(lll.LLLError):
        lll.philox(np.zeros((0, 4), np.uint32), np.zeros((0, 2), np.uint32))
    # the sampler routines reject arguments outside their domains on the host
    for routine, x in (("log", [0.5, 0.0]), ("log", [1.5]), ("log", [1e-310]), ("log", [np.nan]),
                       ("sinpi", [2.5]), ("cospi", [-0.25]), ("sinpi", [0.3]),
                       ("sqrt", [0.0]), ("sqrt", [-1.0]), ("sqrt", [np.inf]),
                       ("div", [[1.0, 0.0]]), ("div", [[1.0, -2.0]]), ("div", [[np.inf, 1.0]])):
        with pytest.raises(lll.LLLError) as ei:
            lll.sampler_math(routine, np.array(x))
        assert ei.value.code == -1, (routine, x)
    lib = lll.load()
    out = np.zeros(1)
    x = np.full(1, 0.5)
    dp = ctypes.POINTER(ctypes.c_double)
    assert lib.lll_sampler_math(5, x.ctypes.data_as(dp), 1, out.ctypes.data_as(dp), None) == -1
    assert lib.lll_sampler_math(0, x.ctypes.data_as(dp), 0, out.ctypes.data_as(dp), None) == -1


def test_batch_validation_errors():
    """Batch arguments are checked on the host before any device work."""
    import paper_1006_3340_amd as lll
    ts = workloads.plain_fp64()
    with pytest.raises(lll.LLLError) as ei:
        lll.Batch([ts], max_paths_each=0)
    assert ei.value.code == -1
    # 4096 structures x 2^30 paths: 2^34 block work items
    with pytest.raises(lll.LLLError) as ei:
        lll.Batch([ts] * 4096, max_paths_each=1 << 30)
    assert ei.value.code == -1 and "work items" in str(ei.value)
    with pytest.raises(lll.LLLError) as ei:
        lll.Batch([ts.copy(L0=-ts.L0)], max_paths_each=64)
    assert ei.value.code == -1
    # the one-shot batch needs its output buffers
    import paper_1006_3340_amd._lib as L
    lib = L.load()
    t = L._TS(ts)
    rc = lib.lll_price_caplets_batched(ctypes.byref(t.c), 1, 64, 0, 1, None, None, None)
    assert rc == -1 and "price_host" in lib.lll_last_error().decode()
    # batches run the 40-slot path kernel: N = 41 is rejected before allocation
    big = workloads.make_structure(41, 0.25, 0.03, 2, lambda t, T, r: 0.1, [1.0])
    with pytest.raises(lll.LLLError) as ei:
        lll.Batch([ts, big], max_paths_each=64)
    assert ei.value.code == -1 and "structure 1" in str(ei.value)


def test_binding_constants_match_the_header():
    """Scheme numbers and size limits of the binding are the header's."""
    import paper_1006_3340_amd as lll
    import paper_1006_3340_amd._lib as L
    text = open(os.path.join(ROOT, "include", "lll.h")).read()
    enum = dict((k, int(v)) for k, v in re.findall(r"\bLLL_([A-Z_0-9]+) = (\d+)", text))
    for name in ("FULL", "PICARD", "FROZEN", "FIRST_ORDER", "SECOND_ORDER", "PICARD_MP", "EXACT",
                 "MLP_DRIFT"):
        assert getattr(L, name) == enum[name], name
        assert lll.SCHEMES[name.lower()] == enum[name], name
    defines = dict((k, int(v)) for k, v in re.findall(r"#define LLL_([A-Z_0-9]+) (\d+)", text))
    assert (L.N_MAX, L.N_MAX_MP, L.N_MAX_FP64, L.N_MAX_EXACT, L.S_MAX, L.Q) == (
        defines["N_MAX"], defines["N_MAX_MP"], defines["N_MAX_FP64"], defines["N_MAX_EXACT"],
        defines["S_MAX"], defines["Q"])


def test_static_workspace_checks_on_the_host():
    """lll_price_caplets_static rejects a pass larger than its static device
    workspace, and the schemes it does not run, before any device call (so
    this runs without a GPU)."""
    import paper_1006_3340_amd as lll
    with pytest.raises(lll.LLLError) as ei:
        lll.price_caplets_static(workloads.learned_drift(), 1 << 20, lll.FULL)
    assert ei.value.code == -1 and "static workspace holds" in str(ei.value)
    with pytest.raises(lll.LLLError) as ei:
        lll.price_caplets_static(workloads.plain_fp64(), 64, lll.PICARD_MP)
    assert ei.value.code == -5
    with pytest.raises(lll.LLLError) as ei:
        lll.price_caplets_static(workloads.plain_fp64().copy(L0=-workloads.plain_fp64().L0), 64)
    assert ei.value.code == -1
