"""Out-of-memory paths through the C ABI.  irs_debug_fail_alloc makes one
chosen device allocation of the library fail, as an exhausted hipMalloc
would: the call must return IRS_E_NOMEM, a failed irs_plan or
irs_batch_create must leave a NULL handle, nothing the failed call allocated
may stay allocated, and a plan or batch that exists must keep working (the
next call without the failure gives the same map as a fresh plan).

What stays allocated is read from the library's own ledger of live device
allocations (irs_debug_live_allocs), exactly: the device's free memory is no
measure of it, since the HIP runtime may keep freed memory for a while."""
import ctypes as C

import numpy as np
import pytest

from gpu_common import Case

pytestmark = pytest.mark.gpu

IRS_E_NOMEM = 3


@pytest.fixture(scope="module")
def irs():
    import paper_2204_10871_amd as irs
    irs.load()
    return irs


def say(msg):
    print(msg, flush=True)


def _live(lib):
    """(count, bytes) of the library's live device allocations."""
    n, b = C.c_int64(-1), C.c_int64(-1)
    assert lib.irs_debug_live_allocs(C.byref(n), C.byref(b)) == 0
    return n.value, b.value


def _case():
    # about 2e5 lenses: every plan buffer is a few MB, so a leaked one shows
    return Case(0.45, 0.05, 0.45, 40.0, 96, n_rays=300_000, n_lens=200_003, seed=61)


def _plan_args(irs, c, method):
    p = irs.make_params(**c.kw, method=method, precision="fp64", **c.p_extra)
    x = np.ascontiguousarray(c.lenses.x, np.float64)
    y = np.ascontiguousarray(c.lenses.y, np.float64)
    return p, x, y


def _plan_cycle(lib, c, p, x, y):
    """irs_plan with each of its allocations failing in turn, then once
    without a failure (freed at once).  Returns the number of failures."""
    k = 0
    while True:
        lib.irs_debug_fail_alloc(k)
        h = C.c_void_p(1)                   # not NULL: the call must clear it
        st = lib.irs_plan(C.byref(p), c.lenses.n, x.ctypes.data, y.ctypes.data, None, None,
                          C.byref(h))
        lib.irs_debug_fail_alloc(-1)
        if st == 0:
            lib.irs_free(h)
            return k
        assert st == IRS_E_NOMEM, (k, st)
        assert h.value is None, k
        assert lib.irs_last_error()                 # a message says what failed
        k += 1
        assert k < 100


@pytest.mark.parametrize("method", ["direct", "interp"])
def test_plan_fails_cleanly_at_every_allocation(irs, method):
    lib = irs._ffi.load()
    c = _case()
    p, x, y = _plan_args(irs, c, method)
    before = _live(lib)
    k = _plan_cycle(lib, c, p, x, y)
    say(f"irs_plan ({method}): {k} allocations failed in turn, live after: {_live(lib)}")
    assert k >= 5
    assert _live(lib) == before


def _map_cycle(irs, lib, c, want):
    """A fresh plan whose first map has each allocation fail in turn, then
    succeed; the map must equal want, also on a second call."""
    k = 0
    with c.plan("interp", "fp64") as pl:
        npix = c.geo.npix
        while True:
            counts = np.zeros(npix * npix, np.uint32)
            st_ = irs.MapStats()
            lib.irs_debug_fail_alloc(k)
            st = lib.irs_shoot_map(pl.handle, counts.ctypes.data, C.byref(st_), 0)
            lib.irs_debug_fail_alloc(-1)
            if st == 0:
                break
            assert st == IRS_E_NOMEM, (k, st)
            k += 1
            assert k < 100
        assert np.array_equal(counts.reshape(npix, npix), want)
        got, _ = pl.shoot_map()
        assert np.array_equal(got, want)
    return k


def test_map_fails_cleanly_and_the_plan_recovers(irs):
    """Each allocation of the first interpolated map (tables, coefficient
    band, expansions, count buffer) fails in turn; the plan then shoots the
    same map as a fresh plan."""
    lib = irs._ffi.load()
    c = _case()
    with c.plan("interp", "fp64") as ref:
        want, _ = ref.shoot_map()
    before = _live(lib)
    k = _map_cycle(irs, lib, c, want)
    say(f"irs_shoot_map: {k} allocations failed in turn, live after: {_live(lib)}")
    assert k >= 3
    assert _live(lib) == before


def _batch_cycle(lib, arr, n):
    k = 0
    while True:
        lib.irs_debug_fail_alloc(k)
        h = C.c_void_p(1)
        st = lib.irs_batch_create(arr, n, None, C.byref(h))
        lib.irs_debug_fail_alloc(-1)
        if st == 0:
            lib.irs_batch_free(h)
            return k
        assert st == IRS_E_NOMEM, (k, st)
        assert h.value is None, k
        k += 1
        assert k < 100


def _small_cases(seed):
    return [Case(0.3, 0.0, 0.3, 8.0, 64, n_rays=100_000 + 977 * i, seed=seed + i)
            for i in range(3)]


@pytest.mark.parametrize("method,precision", [("direct", "fp32"), ("interp", "fp64")])
def test_batch_create_fails_cleanly(irs, method, precision):
    lib = irs._ffi.load()
    before = _live(lib)
    plans = [cc.plan(method, precision) for cc in _small_cases(70)]
    try:
        with_plans = _live(lib)
        arr = (C.c_void_p * len(plans))(*[pl.handle.value for pl in plans])
        k = _batch_cycle(lib, arr, len(plans))
        say(f"irs_batch_create ({method}): {k} allocations failed in turn")
        assert k >= 1
        assert _live(lib) == with_plans
    finally:
        for pl in plans:
            pl.close()
    assert _live(lib) == before


def test_batch_run_fails_cleanly_and_recovers(irs):
    """Each allocation of an interpolated batch's first run (every map's
    whole-map level-2 buffers and tables) fails in turn; the run that
    follows gives every map as its plan alone does, and freeing the batch
    and plans leaves nothing allocated."""
    import torch
    lib = irs._ffi.load()
    cases = _small_cases(80)
    want = []
    for cc in cases:
        with cc.plan("interp", "fp64") as pl:
            want.append(pl.shoot_map()[0])
    before = _live(lib)
    plans = [cc.plan("interp", "fp64") for cc in cases]
    try:
        with irs.Batch(plans) as b:
            info = b.info()
            assert info["whole_maps"] == 1, info
            counts = [torch.empty(cc.geo.npix ** 2, dtype=torch.int32, device="cuda:0")
                      for cc in cases]
            ptrs = (C.c_void_p * len(counts))(*[t.data_ptr() for t in counts])
            k = 0
            while True:
                lib.irs_debug_fail_alloc(k)
                st = lib.irs_batch_run(b._h, ptrs, None, 0)
                lib.irs_debug_fail_alloc(-1)
                if st == 0:
                    break
                assert st == IRS_E_NOMEM, (k, st)
                k += 1
                assert k < 200
            torch.cuda.synchronize()
            say(f"irs_batch_run: {k} allocations failed in turn")
            assert k >= 3
            for cc, t, w in zip(cases, counts, want):
                got = t.cpu().numpy().view(np.uint32).reshape(cc.geo.npix, cc.geo.npix)
                assert np.array_equal(got, w)
            assert lib.irs_batch_run(b._h, ptrs, None, 0) == 0          # the graph replays
            torch.cuda.synchronize()
            for cc, t, w in zip(cases, counts, want):
                got = t.cpu().numpy().view(np.uint32).reshape(cc.geo.npix, cc.geo.npix)
                assert np.array_equal(got, w)
    finally:
        for pl in plans:
            pl.close()
    assert _live(lib) == before
