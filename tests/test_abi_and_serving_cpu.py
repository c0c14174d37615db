"""Host-side checks that need no GPU: the C ABI library loads and exports
every function include/fmm.h declares, and the serving scheduler (admission
by footprint, arrival order, slot limit, errors and time-outs) behaves as
specified, driven through a device-less context whose executor only waits a
simulated time."""
import os
import re
import time

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "fmm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(fmm_\w+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_symbol():
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2005_12351_amd", "libfmm.so"))
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_declared_symbols():
    from paper_2005_12351_amd import fmm
    for n in _declared():
        assert n in fmm.EXPORTED, n


@pytest.fixture
def fmm():
    from paper_2005_12351_amd import fmm as f
    return f


def _req(ctx, n, p=4, order=0, **kw):
    return ctx.submit(n=n, order=order, p=p, theta=0.5, ncrit=64, **kw)


def test_fake_server_completes_in_order(fmm):
    ctx = fmm.Context.fake(budget_bytes=1 << 40, ns_per_particle=2000.0)
    ctx.serve_start(3)
    tickets = [_req(ctx, 1000 + 100 * k) for k in range(10)]
    for t in tickets:
        ctx.wait(t, 10.0)
        assert ctx.poll(t) == fmm.FMM_REQ_DONE
    times = [ctx.request_times(t) for t in tickets]
    admits = [x["admit"] for x in times]
    assert admits == sorted(admits)                      # arrival order
    assert all(x["submit"] <= x["admit"] <= x["done"] for x in times)
    st = ctx.serve_stats()
    assert st["peak_running"] == 3 and st["in_use"] == 0 and st["queued"] == 0
    ctx.close()


def test_fake_server_admission_by_footprint(fmm):
    # budget fits two of these requests at a time, whatever the slot count
    probe = fmm.Context.fake(budget_bytes=1 << 40)
    probe.serve_start(1)
    one = probe.request_times(_req(probe, 200_000))["footprint"]
    probe.close()
    ctx = fmm.Context.fake(budget_bytes=int(2.5 * one), ns_per_particle=200.0)
    ctx.serve_start(8)
    tickets = [_req(ctx, 200_000) for _ in range(6)]
    for t in tickets:
        ctx.wait(t, 20.0)
    st = ctx.serve_stats()
    assert st["peak_running"] == 2
    assert st["peak_in_use"] <= st["budget"]
    ctx.close()


def test_fake_server_rejections_and_timeout(fmm):
    ctx = fmm.Context.fake(budget_bytes=64 << 20, ns_per_particle=1e6)
    with pytest.raises(fmm.FMMError) as e:
        _req(ctx, 1000)                                 # not started
    assert e.value.code == fmm.FMM_ESTATE
    ctx.serve_start(1)
    with pytest.raises(fmm.FMMError) as e:
        _req(ctx, 50_000_000)                           # can never fit
    assert e.value.code == fmm.FMM_ENOMEM
    with pytest.raises(fmm.FMMError) as e:
        _req(ctx, 1000, p=0)                            # p < order + 1
    assert e.value.code == fmm.FMM_EINVAL
    with pytest.raises(fmm.FMMError) as e:
        ctx.submit(n=100, order=1, p=4, theta=1.5, ncrit=8)
    assert e.value.code == fmm.FMM_EINVAL
    t = _req(ctx, 2000)                                 # 2 ms simulated
    with pytest.raises(fmm.FMMError) as e:
        ctx.wait(t, 0.0)
    assert e.value.code == fmm.FMM_ETIMEOUT
    ctx.wait(t, 10.0)
    assert ctx.poll(t) == fmm.FMM_REQ_DONE
    with pytest.raises(fmm.FMMError):
        ctx.poll(987654)
    ctx.close()


def test_fake_server_stop_drains_queue(fmm):
    ctx = fmm.Context.fake(budget_bytes=1 << 40, ns_per_particle=500.0)
    ctx.serve_start(2)
    tickets = [_req(ctx, 4000) for _ in range(8)]
    t0 = time.time()
    ctx.serve_stop()
    assert time.time() - t0 < 10.0
    # the server is gone; the context can start a new one
    ctx.serve_start(1)
    t = _req(ctx, 10)
    ctx.wait(t, 5.0)
    ctx.close()
    assert len(tickets) == 8


def test_overlap_modes_validated(fmm):
    """fmm_ctx_set_overlap takes FMM_OVERLAP_OFF / WHOLE / SPLIT / TAIL and
    rejects anything else with FMM_EINVAL (no device needed)"""
    ctx = fmm.Context.fake(budget_bytes=1 << 30)
    for mode in (fmm.FMM_OVERLAP_OFF, fmm.FMM_OVERLAP_WHOLE, fmm.FMM_OVERLAP_SPLIT, fmm.FMM_OVERLAP_TAIL, False, True):
        ctx.set_overlap(mode)
    for bad in (-1, 4):
        with pytest.raises(RuntimeError, match="overlap mode"):
            ctx.set_overlap(bad)
    ctx.close()
