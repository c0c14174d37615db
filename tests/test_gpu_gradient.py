"""GPU parity of the field gradient (fmm_evaluate_grad) against the oracle's
gradient on the same tree, lists and truncation: for FMM the second
derivatives of the local expansion plus the near-field pairs' closed forms,
for Barnes-Hut the second derivatives of each accepted cell's M2P plus the
pairs of the unaccepted leaves.

Tolerances (relative L2 over all targets and the six components):
- FP64: 1e-10, as for phi and E (same arithmetic up to summation order).
- MIXED: 2e-6.  The gradient is dominated by the near field, whose pair
  terms are FP32: a few units of roundoff (6e-8) each, with cancellation
  between the delta and r_i r_j parts (up to 3x for a charge, more for the
  quadrupole's five terms) and Kahan-compensated sums; the far part comes
  from the FP32 M2L like the field's.  Observed: 2.1e-7 to 5.6e-7 (FP64
  4e-16 to 3e-15); the values are printed.
Largest per-target error (tests/gpu_helpers.py): FP64 1e-12 as for phi and
E; MIXED 1e-4, since a target's gradient is dominated by its nearest pairs,
whose r^-3 and r^-5 terms cancel most among the outputs.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2005_12351_amd import fmm  # noqa: E402
from paper_2005_12351_amd import workloads as W  # noqa: E402
from tests.gpu_helpers import PHI_FLOOR, rel_l2, to_dev, within  # noqa: E402

TOL = {fmm.FMM_PREC_FP64: (1e-10, 1e-12), fmm.FMM_PREC_MIXED: (2e-6, 1e-4)}
ALL = fmm.FMM_POT | fmm.FMM_FIELD | fmm.FMM_GRAD


@pytest.fixture(scope="module")
def ctx():
    c = fmm.Context(0)
    yield c
    c.close()


def _gpu_grad(ctx, w, prec, outputs=ALL):
    t = fmm.Tree(ctx, to_dev(w.pos), w.ncrit, w.theta)
    t.upward(w.order, to_dev(w.moments), w.p, prec)
    ph, E, G = t.evaluate_grad(outputs)
    torch.cuda.synchronize()
    out = tuple(None if x is None else x.cpu().numpy() for x in (ph, E, G))
    return out, t


# (order code, p, kind, n, ncrit, theta); p - s = 2 is the smallest allowed
CASES = [(0, 4, "uniform", 2000, 32, 0.5), (1, 8, "uniform", 3000, 32, 0.5), (2, 10, "lattice", 3375, 64, 0.5),
         (1, 6, "plummer", 4000, 32, 0.6), (0, 2, "uniform", 1500, 16, 0.5), (1, 3, "plummer", 2500, 8, 0.4),
         (2, 4, "uniform", 1200, 16, 0.5)]


@pytest.mark.parametrize("order,p,kind,n,ncrit,theta", CASES)
@pytest.mark.parametrize("prec", [fmm.FMM_PREC_FP64, fmm.FMM_PREC_MIXED])
def test_gradient_matches_oracle(orc, ctx, order, p, kind, n, ncrit, theta, prec):
    print(f"[grad] order={order} p={p} {kind} n={n} ncrit={ncrit} theta={theta} precision={prec}", flush=True)
    w = W.small_random(1300 + n + order, n, order, kind, p=p, theta=theta, ncrit=ncrit)
    (ph, E, G), t = _gpu_grad(ctx, w, prec)
    t.close()
    po, Eo, Go = orc.Tree(w.pos, ncrit, theta).fmm(order, w.moments, p, want_grad=True)
    ok = within(G, Go, prec, "G vs oracle", TOL[prec])
    ok &= within(ph, po, prec, "phi vs oracle", floor=PHI_FLOOR)
    ok &= within(E, Eo, prec, "E vs oracle")
    assert ok
    assert np.abs(G[:, 0] + G[:, 3] + G[:, 5]).max() <= 1e-5 * np.abs(G).max()   # Laplace: trace ~ 0


@pytest.mark.parametrize("mask,p", [(7, 6), (6, 5), (3, 4)])
@pytest.mark.parametrize("prec", [fmm.FMM_PREC_FP64, fmm.FMM_PREC_MIXED])
def test_gradient_mixed_orders(orc, ctx, mask, p, prec):
    w = W.small_mixed(1400 + mask, 2500, mask, "plummer", p=p, theta=0.5, ncrit=32)
    print(f"[grad mixed] mask={mask} p={p} precision={prec}", flush=True)
    (_, _, G), t = _gpu_grad(ctx, w, prec)
    t.close()
    Go = orc.Tree(w.pos, w.ncrit, w.theta).fmm(w.order, w.moments, p, want_grad=True)[2]
    assert within(G, Go, prec, "G vs oracle", TOL[prec])


@pytest.mark.parametrize("basis", [fmm.FMM_M2L_HARMONIC, fmm.FMM_M2L_FULL])
@pytest.mark.parametrize("prec", [fmm.FMM_PREC_FP64, fmm.FMM_PREC_MIXED])
def test_gradient_keeps_phi_field_and_replays(ctx, basis, prec):
    """phi and E from fmm_evaluate_grad are bit-identical to fmm_evaluate's;
    replays of the captured sequence (eager work and synchronisations in
    between) reproduce the gradient exactly."""
    w = W.small_random(1500, 5000, 1, "plummer", p=7, theta=0.5, ncrit=32)
    ctx.set_m2l_basis(basis)
    try:
        t = fmm.Tree(ctx, to_dev(w.pos), w.ncrit, w.theta)
        mom = to_dev(w.moments)
        t.upward(w.order, mom, w.p, prec)
        ph0, E0 = t.evaluate()
        phi = torch.empty(w.n, dtype=torch.float64, device="cuda")
        fld = torch.empty((w.n, 3), dtype=torch.float64, device="cuda")
        grd = torch.empty((w.n, 6), dtype=torch.float64, device="cuda")
        ref = None
        for rep in range(4):
            for x in (phi, fld, grd):
                x.fill_(float("nan"))
            t.evaluate_grad(ALL, phi, fld, grd)
            torch.cuda.synchronize()
            assert np.isfinite((to_dev(w.pos) * 2.0).sum().item())     # eager work between replays
            assert torch.equal(phi, ph0) and torch.equal(fld, E0), rep
            g = grd.cpu().numpy()
            if ref is None:
                ref = g
            assert np.array_equal(g, ref), rep
        # the gradient alone, then a plain evaluate again: both unchanged
        _, _, g2 = t.evaluate_grad(fmm.FMM_GRAD)
        ph3, E3 = t.evaluate()
        torch.cuda.synchronize()
        assert np.array_equal(g2.cpu().numpy(), ref) and torch.equal(ph3, ph0) and torch.equal(E3, E0)
        t.close()
    finally:
        ctx.set_m2l_basis(fmm.FMM_M2L_HARMONIC)


@pytest.mark.parametrize("index", [2, 3])
def test_gradient_full_size_sampled(orc, ctx, index):
    """100k uniform dipoles, p 8 (the benchmark workload; L2P keeps the
    locals as cubes) and 1M Plummer dipoles, p 6 (enough L2P waves that it
    keeps them as packed columns), after fmm_run, on 4 096 sampled targets."""
    w = W.config(index)
    print(f"[grad full] {w.name}", flush=True)
    Go = orc.Tree(w.pos, w.ncrit, w.theta).fmm(w.order, w.moments, w.p, targets=w.sample, want_grad=True)[2]
    t = fmm.Tree(ctx, to_dev(w.pos), w.ncrit, w.theta)
    s = torch.from_numpy(w.sample).cuda()
    outputs = fmm.FMM_FIELD if w.outputs == "field" else (fmm.FMM_POT | fmm.FMM_FIELD)
    for prec in (fmm.FMM_PREC_FP64, fmm.FMM_PREC_MIXED):
        t.run(w.order, to_dev(w.moments), w.p, prec, outputs)
        _, _, G = t.evaluate_grad(fmm.FMM_GRAD)
        torch.cuda.synchronize()
        assert within(G[s].cpu().numpy(), Go, prec, f"precision={prec}: G vs oracle", TOL[prec])
    t.close()


def test_gradient_errors(ctx):
    w = W.small_random(1600, 800, 1, "uniform", p=2, theta=0.5, ncrit=16)
    pos, mom = to_dev(w.pos), to_dev(w.moments)
    t = fmm.Tree(ctx, pos, w.ncrit, w.theta)
    with pytest.raises(RuntimeError):
        t.evaluate_grad(fmm.FMM_GRAD)                      # before fmm_upward: FMM_ESTATE
    t.upward(1, mom, 2, fmm.FMM_PREC_FP64)
    with pytest.raises(RuntimeError, match="p - s >= 2"):
        t.evaluate_grad(fmm.FMM_GRAD)                      # p - s = 1
    t.upward(1, mom, 3, fmm.FMM_PREC_FP64)
    g = torch.empty((w.n, 6), dtype=torch.float64, device="cuda")
    t.evaluate_grad(fmm.FMM_GRAD, None, None, g)           # p - s = 2 works
    with pytest.raises(RuntimeError):
        fmm._check(fmm.fmm_evaluate_grad(ctx.h, t.h, fmm.FMM_GRAD, None, None, None), "fmm_evaluate_grad")
    with pytest.raises(RuntimeError):
        fmm._check(fmm.fmm_evaluate(ctx.h, t.h, fmm.FMM_GRAD, None, None), "fmm_evaluate")
    t.close()
    tb = fmm.Tree(ctx, pos, w.ncrit, w.theta, fmm.FMM_METHOD_BH)
    with pytest.raises(RuntimeError):
        tb.evaluate_grad(fmm.FMM_GRAD)                     # BH before fmm_upward: FMM_ESTATE
    tb.upward(1, mom, 1, fmm.FMM_PREC_FP64)
    tb.evaluate_grad(fmm.FMM_GRAD, None, None, g)          # BH: no p - s restriction
    with pytest.raises(RuntimeError):
        fmm._check(fmm.fmm_evaluate_grad(ctx.h, tb.h, fmm.FMM_GRAD, None, None, None), "fmm_evaluate_grad")
    tb.close()


# Barnes-Hut: accepted cells through the second derivatives of the M2P,
# unaccepted leaves through the pairs' closed forms, against the oracle's
# traversal on the same tree (same acceptance decisions, taken in FP64).
BH_CASES = [(1, 6, "plummer", 4000, 32, 0.6), (0, 4, "uniform", 3000, 16, 0.5), (2, 5, "lattice", 3375, 64, 0.4),
            (1, 1, "plummer", 3000, 16, 0.5), (2, 2, "uniform", 1000, 8, 0.6), (0, 10, "uniform", 700, 4, 0.5)]
BASES = {"harmonic": fmm.FMM_M2L_HARMONIC, "full": fmm.FMM_M2L_FULL}


def _bh_grad(ctx, w, p, theta, ncrit, prec, basis, outputs=ALL):
    ctx.set_m2l_basis(BASES[basis])
    try:
        t = fmm.Tree(ctx, to_dev(w.pos), ncrit, theta, fmm.FMM_METHOD_BH)
        t.upward(w.order, to_dev(w.moments), p, prec)
        out = t.evaluate_grad(outputs)
        ref = t.evaluate(outputs & (fmm.FMM_POT | fmm.FMM_FIELD)) if outputs & 3 else (None, None)
        torch.cuda.synchronize()
        t.close()
    finally:
        ctx.set_m2l_basis(fmm.FMM_M2L_HARMONIC)
    cpu = lambda x: None if x is None else x.cpu().numpy()   # noqa: E731
    return tuple(cpu(x) for x in out), tuple(cpu(x) for x in ref)


@pytest.mark.parametrize("order,p,kind,n,ncrit,theta", BH_CASES)
@pytest.mark.parametrize("prec", [fmm.FMM_PREC_FP64, fmm.FMM_PREC_MIXED])
@pytest.mark.parametrize("basis", list(BASES))
def test_bh_gradient_matches_oracle(orc, ctx, order, p, kind, n, ncrit, theta, prec, basis):
    print(f"[bh grad {basis}] order={order} p={p} {kind} n={n} ncrit={ncrit} theta={theta} precision={prec}",
          flush=True)
    w = W.small_random(1700 + n + order, n, order, kind)
    (ph, E, G), (ph0, E0) = _bh_grad(ctx, w, p, theta, ncrit, prec, basis)
    po, Eo, Go = orc.Tree(w.pos, ncrit).bh(order, w.moments, p, theta, want_grad=True)
    print(f"   vs fmm_evaluate: phi {rel_l2(ph, ph0):.1e} E {rel_l2(E, E0):.1e}", flush=True)
    assert within(G, Go, prec, "G vs oracle BH", TOL[prec])
    # phi and E of the gradient variant agree with the plain traversal's to
    # rounding: the two kernels are compiled apart and the FP32 M2P may round
    # in another order (observed 5e-9 MIXED, 3e-17 FP64)
    agree = 1e-14 if prec == fmm.FMM_PREC_FP64 else 1e-7
    assert rel_l2(ph, ph0) < agree and rel_l2(E, E0) < agree
    ok = within(ph, po, prec, "phi vs oracle BH", floor=PHI_FLOOR)
    ok &= within(E, Eo, prec, "E vs oracle BH")
    assert ok
    assert np.abs(G[:, 0] + G[:, 3] + G[:, 5]).max() <= 1e-5 * np.abs(G).max()


@pytest.mark.parametrize("mask,p", [(7, 6), (5, 3)])
@pytest.mark.parametrize("prec", [fmm.FMM_PREC_FP64, fmm.FMM_PREC_MIXED])
def test_bh_gradient_mixed_orders(orc, ctx, mask, p, prec):
    w = W.small_mixed(1800 + mask, 2500, mask, "plummer", p=p, theta=0.5, ncrit=32)
    print(f"[bh grad mixed] mask={mask} p={p} precision={prec}", flush=True)
    (_, _, G), _ = _bh_grad(ctx, w, p, 0.5, 32, prec, "harmonic", fmm.FMM_GRAD)
    Go = orc.Tree(w.pos, 32).bh(w.order, w.moments, p, 0.5, want_grad=True)[2]
    assert within(G, Go, prec, "G vs oracle BH", TOL[prec])


def test_bh_gradient_full_size_sampled(orc, ctx):
    """1M Plummer dipoles, p 6, theta 0.6 (the Barnes-Hut benchmark workload)
    after fmm_run, on 4 096 sampled targets, both precisions"""
    w = W.config(3)
    print(f"[bh grad full] {w.name}", flush=True)
    Go = orc.Tree(w.pos, w.ncrit).bh(w.order, w.moments, w.p, w.theta, targets=w.sample, want_grad=True)[2]
    t = fmm.Tree(ctx, to_dev(w.pos), w.ncrit, w.theta, fmm.FMM_METHOD_BH)
    s = torch.from_numpy(w.sample).cuda()
    for prec in (fmm.FMM_PREC_FP64, fmm.FMM_PREC_MIXED):
        t.run(w.order, to_dev(w.moments), w.p, prec, fmm.FMM_FIELD)
        _, _, G = t.evaluate_grad(fmm.FMM_GRAD)
        torch.cuda.synchronize()
        assert within(G[s].cpu().numpy(), Go, prec, f"precision={prec}: G vs oracle BH", TOL[prec])
    t.close()


def test_bh_gradient_degenerate(orc, ctx):
    """one particle: no source, zero gradient; two: the pair's closed form"""
    for n in (1, 2, 40):
        w = W.small_random(1900 + n, n, 2, "uniform")
        (_, _, G), _ = _bh_grad(ctx, w, 3, 0.5, 4, fmm.FMM_PREC_FP64, "harmonic", fmm.FMM_GRAD)
        Go = orc.Tree(w.pos, 4).bh(2, w.moments, 3, 0.5, want_grad=True)[2]
        if n == 1:
            assert np.all(G == 0.0)
        else:
            assert within(G, Go, "fp64", f"n={n} G vs oracle BH", TOL[fmm.FMM_PREC_FP64])
