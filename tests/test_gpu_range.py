"""GPU parity far from unit scale: the paper's own timing workload (random
charges in [-1e-9, 1e-9]^3, theta 0.3, ncrit 128, Section 4) at a size the
oracle evaluates in full, the same box for dipoles and quadrupoles, and a box
of side 2e9.  The field of an order-s source scales as r^-(s+2), so in a
1e-9 box a quadrupole's field is ~1e45 and in a 1e9 box ~1e-36: beyond or at
the edge of FP32's range (3.4e38 down to 1.2e-38 normal).  The mixed path
must still meet the FP32 tolerance, which holds only if every FP32 quantity is
kept in cell-relative units (multipoles divided by r^|m|, locals multiplied by
r^(|n|+1), pair separations in units of the leaf radius) and the physical
scale is restored in FP64."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2005_12351_amd import fmm  # noqa: E402
from paper_2005_12351_amd import workloads as W  # noqa: E402
from tests.gpu_helpers import PHI_FLOOR, gpu_fmm, within  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = fmm.Context(0)
    yield c
    c.close()


def _box(half, n, order, seed):
    """n sources of the given order uniform in [-half, half]^3"""
    rng = np.random.default_rng(seed)
    pos = np.ascontiguousarray(rng.uniform(-half, half, (n, 3)))
    mom = W.random_moments(rng, order, n)
    return W.Workload(f"box{half:g}-m{order}", pos, order, mom, 8, 0.3, 128, "pot+field")


# (half side, order, p, theta, ncrit, n): C0 of the paper at n = 5 000, the
# same box with dipoles and quadrupoles, a 1e9 box
CASES = [(1e-9, 0, 8, 0.3, 128, 5000), (1e-9, 1, 8, 0.3, 128, 5000), (1e-9, 2, 8, 0.4, 64, 4000),
         (1e9, 0, 8, 0.3, 128, 5000), (1e9, 1, 6, 0.5, 32, 4000), (1e9, 2, 8, 0.4, 64, 4000)]


@pytest.mark.parametrize("half,order,p,theta,ncrit,n", CASES)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fmm_extreme_box(orc, ctx, half, order, p, theta, ncrit, n, prec):
    w = _box(half, n, order, 4000 + order + (0 if half < 1 else 10))
    print(f"[range fmm] half side {half:g} order={order} p={p} theta={theta} ncrit={ncrit} n={n} {prec}", flush=True)
    pr = fmm.FMM_PREC_FP64 if prec == "fp64" else fmm.FMM_PREC_MIXED
    ph, E, t = gpu_fmm(fmm, ctx, w, p=p, theta=theta, ncrit=ncrit, precision=pr)
    t.close()
    po, Eo = orc.Tree(w.pos, ncrit, theta).fmm(order, w.moments, p)
    assert np.all(np.isfinite(ph)) and np.all(np.isfinite(E))
    ok = within(ph, po, prec, "phi vs oracle FMM", floor=PHI_FLOOR)
    ok &= within(E, Eo, prec, "E vs oracle FMM")
    assert ok


@pytest.mark.parametrize("half,order", [(1e-9, 2), (1e9, 2), (1e-9, 1)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_bh_extreme_box(orc, ctx, half, order, prec):
    w = _box(half, 3000, order, 4100 + order + (0 if half < 1 else 10))
    print(f"[range bh] half side {half:g} order={order} {prec}", flush=True)
    pr = fmm.FMM_PREC_FP64 if prec == "fp64" else fmm.FMM_PREC_MIXED
    ph, E, t = gpu_fmm(fmm, ctx, w, p=6, theta=0.4, ncrit=32, precision=pr, method=fmm.FMM_METHOD_BH)
    t.close()
    po, Eo = orc.Tree(w.pos, 32).bh(order, w.moments, 6, 0.4)
    assert np.all(np.isfinite(ph)) and np.all(np.isfinite(E))
    ok = within(ph, po, prec, "phi vs oracle BH", floor=PHI_FLOOR)
    ok &= within(E, Eo, prec, "E vs oracle BH")
    assert ok
