"""GPU serving: requests of different size, source order, expansion order and
precision run concurrently through the continuous-batching server; each
result must equal the same request evaluated alone (the kernels are
deterministic, so the comparison is exact), and one of them is checked against
the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2005_12351_amd import fmm  # noqa: E402
from paper_2005_12351_amd import workloads as W  # noqa: E402
from tests.gpu_helpers import rel_l2  # noqa: E402


def _mix():
    out = []
    specs = [(3000, 0, 4, "uniform", fmm.FMM_PREC_MIXED), (20000, 1, 6, "plummer", fmm.FMM_PREC_MIXED),
             (8000, 2, 8, "uniform", fmm.FMM_PREC_FP64), (50000, 1, 8, "uniform", fmm.FMM_PREC_MIXED),
             (1000, 0, 6, "plummer", fmm.FMM_PREC_FP64), (12000, 2, 4, "lattice", fmm.FMM_PREC_MIXED),
             (30000, 0, 8, "plummer", fmm.FMM_PREC_MIXED), (5000, 1, 4, "uniform", fmm.FMM_PREC_FP64),
             (15000, 1, 8, "plummer", fmm.FMM_PREC_MIXED), (2000, 2, 6, "uniform", fmm.FMM_PREC_MIXED)]
    for k, (n, order, p, kind, prec) in enumerate(specs):
        w = W.small_random(3000 + k, n, order, kind, p=p, theta=0.5, ncrit=64)
        out.append((w, prec))
    return out


def test_results_alone_equal_results_in_mix(orc):
    mix = _mix()
    dev = []
    for w, prec in mix:
        dev.append(dict(pos=torch.from_numpy(w.pos).cuda(), mom=torch.from_numpy(w.moments).cuda(),
                        phi=torch.full((w.n,), float("nan"), dtype=torch.float64, device="cuda"),
                        E=torch.full((w.n, 3), float("nan"), dtype=torch.float64, device="cuda")))
    # alone: one request at a time through the direct API
    alone = []
    ctx0 = fmm.Context(0)
    for (w, prec), d in zip(mix, dev):
        t = fmm.Tree(ctx0, d["pos"], w.ncrit, w.theta)
        t.upward(w.order, d["mom"], w.p, prec)
        phi, E = t.evaluate()
        torch.cuda.synchronize()
        alone.append((phi.cpu().numpy(), E.cpu().numpy()))
        t.close()
    ctx0.close()
    # in the mix: all submitted at once to a 4-slot server
    ctx = fmm.Context(0, budget_bytes=4 << 30)
    ctx.serve_start(4)
    tickets = [ctx.submit(n=w.n, order=w.order, p=w.p, theta=w.theta, ncrit=w.ncrit, pos=d["pos"],
                          moments=d["mom"], phi=d["phi"], field=d["E"], precision=prec)
               for (w, prec), d in zip(mix, dev)]
    for t in tickets:
        ctx.wait(t, 60.0)
    st = ctx.serve_stats()
    print("serve stats", st, flush=True)
    assert st["peak_running"] >= 2            # requests really overlapped
    for (a_phi, a_E), d in zip(alone, dev):
        assert np.array_equal(d["phi"].cpu().numpy(), a_phi)
        assert np.array_equal(d["E"].cpu().numpy(), a_E)
    for t in tickets:
        tm = ctx.request_times(t)
        assert tm["submit"] <= tm["admit"] <= tm["done"] and tm["bytes_used"] > 0
    ctx.close()
    # and one of them against the oracle
    w, prec = mix[1]
    po, Eo = orc.Tree(w.pos, w.ncrit, w.theta).fmm(w.order, w.moments, w.p)
    assert rel_l2(alone[1][0], po) < 1e-6 and rel_l2(alone[1][1], Eo) < 1e-6


def test_budget_limits_concurrency():
    ctx = fmm.Context(0, budget_bytes=300 << 20)
    ctx.serve_start(8)
    ws = [W.small_random(9000 + k, 100_000, 1, "uniform", p=6) for k in range(4)]
    dev = [(torch.from_numpy(w.pos).cuda(), torch.from_numpy(w.moments).cuda(),
            torch.empty(w.n, dtype=torch.float64, device="cuda"),
            torch.empty((w.n, 3), dtype=torch.float64, device="cuda")) for w in ws]
    tickets = [ctx.submit(n=w.n, order=1, p=6, theta=0.5, ncrit=64, pos=d[0], moments=d[1], phi=d[2], field=d[3])
               for w, d in zip(ws, dev)]
    for t in tickets:
        ctx.wait(t, 60.0)
    st = ctx.serve_stats()
    fp = ctx.request_times(tickets[0])["footprint"]
    assert st["peak_in_use"] <= st["budget"]
    assert st["peak_running"] <= max(1, st["budget"] // fp)
    ctx.close()
