"""GPU parity of the multipolar Barnes-Hut path (Section 3.2, Eq. 12, Eq. 6)
against the oracle's per-particle traversal on the same tree.  The GPU takes
every acceptance decision in FP64 with the definition's rounding sequence, so
the FP64 path matches the oracle to rounding; the mixed path (FP32 M2P and
direct sums) to the FP32 tolerance."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2005_12351_amd import fmm  # noqa: E402
from paper_2005_12351_amd import workloads as W  # noqa: E402
from tests.gpu_helpers import PHI_FLOOR, gpu_fmm, within  # noqa: E402

# tolerances: those of the FMM (tests/gpu_helpers.py); the mixed path's M2P
# and direct terms are FP32 as the FMM's M2L and P2P


@pytest.fixture(scope="module")
def ctx():
    c = fmm.Context(0)
    yield c
    c.close()


BH_CASES = [(1, 6, "plummer", 5000, 32, 0.6), (1, 6, "plummer", 5000, 32, 0.3), (0, 4, "uniform", 3000, 16, 0.5),
            (2, 5, "lattice", 3375, 64, 0.4), (1, 1, "plummer", 4000, 16, 0.5), (2, 2, "uniform", 1000, 8, 0.6),
            (0, 10, "uniform", 700, 4, 0.5)]


BASES = {"harmonic": fmm.FMM_M2L_HARMONIC, "full": fmm.FMM_M2L_FULL}


@pytest.mark.parametrize("order,p,kind,n,ncrit,theta", BH_CASES)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("basis", list(BASES))
def test_bh_matches_oracle(orc, ctx, order, p, kind, n, ncrit, theta, prec, basis):
    print(f"[bh {prec} {basis}] order={order} p={p} {kind} n={n} ncrit={ncrit} theta={theta}", flush=True)
    w = W.small_random(1200 + n + order, n, order, kind)
    pr = fmm.FMM_PREC_FP64 if prec == "fp64" else fmm.FMM_PREC_MIXED
    ctx.set_m2l_basis(BASES[basis])
    try:
        ph, E, _ = gpu_fmm(fmm, ctx, w, p=p, theta=theta, ncrit=ncrit, precision=pr, method=fmm.FMM_METHOD_BH)
    finally:
        ctx.set_m2l_basis(fmm.FMM_M2L_HARMONIC)
    po, Eo = orc.Tree(w.pos, ncrit).bh(order, w.moments, p, theta)
    ok = within(ph, po, prec, "phi vs oracle BH", floor=PHI_FLOOR)
    ok &= within(E, Eo, prec, "E vs oracle BH")
    assert ok


def test_bh_field_only_and_degenerate(orc, ctx):
    for n in (1, 2, 50):
        w = W.small_random(77 + n, n, 1, "uniform")
        _, E, _ = gpu_fmm(fmm, ctx, w, p=3, theta=0.5, ncrit=4, precision=fmm.FMM_PREC_FP64,
                          method=fmm.FMM_METHOD_BH, outputs=fmm.FMM_FIELD)
        _, Eo = orc.Tree(w.pos, 4).bh(1, w.moments, 3, 0.5)
        if n == 1:
            assert np.all(E == 0.0)
        else:
            assert within(E, Eo, "fp64", f"n={n} E vs oracle BH")
