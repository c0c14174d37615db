"""GPU test of fmm_evaluate_grad_noalloc, the allocation-free variant of
fmm_evaluate_grad: on a fresh tree it holds no more device memory after the
call than before, and its phi, field and gradient equal those of
fmm_evaluate_grad (same kernels, same inputs: bit for bit), on two calls in a
row, the second with a smaller system, in both precisions; Barnes-Hut trees
too; a system beyond the scratch's capacity is refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2005_12351_amd import fmm  # noqa: E402
from paper_2005_12351_amd import workloads as W  # noqa: E402
from tests.gpu_helpers import to_dev  # noqa: E402

ALL = fmm.FMM_POT | fmm.FMM_FIELD | fmm.FMM_GRAD


@pytest.fixture(scope="module")
def ctx():
    c = fmm.Context(0)
    yield c
    c.close()


def _outs(n):
    return (torch.full((n,), float("nan"), dtype=torch.float64, device="cuda"),
            torch.full((n, 3), float("nan"), dtype=torch.float64, device="cuda"),
            torch.full((n, 6), float("nan"), dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("method", [fmm.FMM_METHOD_FMM, fmm.FMM_METHOD_BH])
@pytest.mark.parametrize("prec", [fmm.FMM_PREC_FP64, fmm.FMM_PREC_MIXED])
def test_noalloc_matches_evaluate_grad(ctx, method, prec):
    for k, (n, order, p, kind) in enumerate(((40000, 1, 7, "plummer"), (6000, 2, 6, "uniform"))):
        print(f"[noalloc] call {k + 1}: method={method} precision={prec} n={n} order={order} p={p} {kind}",
              flush=True)
        w = W.small_random(7700 + k, n, order, kind, p=p, theta=0.5, ncrit=32)
        t = fmm.Tree(ctx, to_dev(w.pos), w.ncrit, w.theta, method)
        t.upward(w.order, to_dev(w.moments), w.p, prec)
        torch.cuda.synchronize()
        held = t.info()["bytes"]
        a = _outs(n)
        t.evaluate_grad_noalloc(ALL, *a)
        torch.cuda.synchronize()
        assert t.info()["bytes"] == held          # nothing allocated for the tree
        b = _outs(n)
        t.evaluate_grad(ALL, *b)
        torch.cuda.synchronize()
        if method == fmm.FMM_METHOD_FMM:
            assert t.info()["bytes"] == held + 48 * n   # the allocating call's near-field gradient buffer
        for x, y in zip(a, b):
            xa, ya = x.cpu().numpy(), y.cpu().numpy()
            assert np.all(np.isfinite(xa))
            assert np.array_equal(xa, ya)
        # the gradient alone, into the same buffers, gives the same gradient
        a[2].fill_(float("nan"))
        t.evaluate_grad_noalloc(fmm.FMM_GRAD, None, None, a[2])
        torch.cuda.synchronize()
        assert torch.equal(a[2], b[2])
        t.close()


def test_noalloc_limits(ctx):
    w = W.small_random(7800, 3000, 1, "uniform", p=5, theta=0.5, ncrit=32)
    t = fmm.Tree(ctx, to_dev(w.pos), w.ncrit, w.theta)
    g = torch.empty((w.n, 6), dtype=torch.float64, device="cuda")
    with pytest.raises(fmm.FMMError) as e:
        t.evaluate_grad_noalloc(fmm.FMM_GRAD, None, None, g)          # before fmm_upward
    assert e.value.code == fmm.FMM_ESTATE
    t.upward(1, to_dev(w.moments), 2, fmm.FMM_PREC_FP64)
    with pytest.raises(fmm.FMMError) as e:
        t.evaluate_grad_noalloc(fmm.FMM_GRAD, None, None, g)          # p - s = 1
    assert e.value.code == fmm.FMM_EINVAL
    t.close()
    n = (1 << 18) + 1
    rng = np.random.default_rng(7801)
    big = fmm.Tree(ctx, to_dev(rng.random((n, 3))), 64, 0.5)
    big.upward(0, to_dev(rng.uniform(-1, 1, n)), 4, fmm.FMM_PREC_MIXED)
    gb = torch.empty((n, 6), dtype=torch.float64, device="cuda")
    with pytest.raises(fmm.FMMError) as e:
        big.evaluate_grad_noalloc(fmm.FMM_GRAD, None, None, gb)       # beyond the scratch
    assert e.value.code == fmm.FMM_EINVAL
    phi = torch.empty(n, dtype=torch.float64, device="cuda")
    big.evaluate_grad_noalloc(fmm.FMM_POT, phi, None, None)           # no gradient: no scratch needed
    ref, _ = big.evaluate(fmm.FMM_POT)
    torch.cuda.synchronize()
    assert torch.equal(phi, ref)
    big.close()
