"""Storage of the expansions per cell: O(p^3) in the full basis, O(p^2) in
the harmonic basis (multipoles kept only as rows folded onto their m_z <= 1
components, locals only as their n_z <= 1 components; the paper's outlook on
irreducible representations).  The device bytes a tree holds must fall by at
least the difference of the two row sizes times the cells, and the two bases
must give the same potentials and fields."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2005_12351_amd import fmm  # noqa: E402
from paper_2005_12351_amd import workloads as W  # noqa: E402
from tests.gpu_helpers import PHI_FLOOR, to_dev, within  # noqa: E402


def nterms(p):
    return 0 if p < 0 else (p + 1) * (p + 2) * (p + 3) // 6


def hterms(p):
    return 0 if p < 0 else (p + 1) ** 2


@pytest.fixture(scope="module")
def ctx():
    c = fmm.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec", [fmm.FMM_PREC_FP64, fmm.FMM_PREC_MIXED])
@pytest.mark.parametrize("method", [fmm.FMM_METHOD_FMM, fmm.FMM_METHOD_BH])
def test_harmonic_basis_stores_reduced_rows(ctx, prec, method):
    w = W.small_random(4100, 30000, 1, "uniform")
    p, s = 10, 1
    print(f"[storage] method={method} precision={prec}", flush=True)
    held, out = {}, {}
    for basis in (fmm.FMM_M2L_FULL, fmm.FMM_M2L_HARMONIC):
        ctx.set_m2l_basis(basis)
        try:
            t = fmm.Tree(ctx, to_dev(w.pos), 32, 0.5, method)
            t.upward(1, to_dev(w.moments), p, prec)
            ph, E = t.evaluate()
            torch.cuda.synchronize()
            info = t.info()
            held[basis] = info["bytes"]
            out[basis] = (ph.cpu().numpy(), E.cpu().numpy())
            nc = info["ncells"]
            t.close()
        finally:
            ctx.set_m2l_basis(fmm.FMM_M2L_HARMONIC)
    # FP64 full rows of the multipoles (and, for FMM, of the locals) give way
    # to folded multipoles and reduced locals; what the bases share aside
    saved_m = nterms(p) - nterms(s - 1) - (hterms(p) - hterms(s - 1))
    saved_l = nterms(p - s) - hterms(p - s) if method == fmm.FMM_METHOD_FMM else 0
    # in MIXED the full basis also keeps an FP32 copy of the full rows, the
    # harmonic one an FP64 state beside its FP32 folded rows
    extra = 0 if prec == fmm.FMM_PREC_FP64 else (nterms(p) - nterms(s - 1)) * 4 - (hterms(p) - hterms(s - 1)) * 4
    bound = nc * (8 * (saved_m + saved_l) + extra)
    print(f"held: full {held[fmm.FMM_M2L_FULL]} harmonic {held[fmm.FMM_M2L_HARMONIC]} bound {bound}")
    assert held[fmm.FMM_M2L_FULL] - held[fmm.FMM_M2L_HARMONIC] >= 0.9 * bound
    pf, Ef = out[fmm.FMM_M2L_FULL]
    ph, Eh = out[fmm.FMM_M2L_HARMONIC]
    # FP64: the same numbers to rounding.  MIXED: two FP32 results, each held
    # to the oracle per target by the parity tests of its basis; between them
    # the pooled bound (their per-target errors need not be alike: at p = 10
    # the FP32 M2P of the two bases rounds differently)
    tol = None if prec == fmm.FMM_PREC_FP64 else (2e-6, 1.0)
    ok = within(ph, pf, prec, "phi harmonic vs full", tol, floor=PHI_FLOOR)
    ok &= within(Eh, Ef, prec, "E harmonic vs full", tol)
    assert ok
