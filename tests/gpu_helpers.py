"""Shared helpers of the GPU parity tests: run the C-ABI library on seeded
inputs and compare with the oracle.

Every comparison checks two things (``within``):
- the relative L2 error over all compared targets (every component pooled);
- the largest per-target error, |a_i - b_i| / max(|b_i|, f rms_j |b_j|),
  with the vector norm of a target's components (E: 3, G: 6), so that a few
  bad targets cannot hide in the pooled norm.  The floor f rms keeps targets
  whose value nearly cancels from dividing by almost nothing: f = 1e-3 for
  the field and its gradient, f = 1 for the potential.  The potential of
  dipoles and quadrupoles cancels far more than the field (its terms fall off
  one power of r more slowly, so far sources of both signs contribute), and
  the rounding error of a target's potential is set by the magnitude of its
  terms, about the rms potential: measured, the largest |a_i - b_i| / rms is
  about 10 u in FP32 and 20 u in FP64 (u the unit roundoff), at targets where
  |b_i| is a thousandth of the rms or less.
"""
import numpy as np
import torch

# (pooled relative L2, largest per-target error) per precision:
# - FP64: both sides compute the same truncated sums (same tree, lists and
#   p) and differ only in summation order and recurrences, a few ulp per
#   coefficient; 1e-12 per target leaves three orders of headroom for the
#   far field's cancellation and still fails on any missing term (>= 1e-6).
# - MIXED: FP32 terms (u = 6e-8) with FP32 per-chunk sums; a target's error
#   relative to its own value is a few u times the ratio of the sum of its
#   terms' magnitudes to the sum, which the 1e-3 floor bounds; 2e-5 per
#   target and 1e-6 pooled.
TOL = {"fp64": (1e-10, 1e-12), "mixed": (1e-6, 2e-5)}
PHI_FLOOR, FIELD_FLOOR = 1.0, 1e-3


def prec_name(prec):
    """'fp64' / 'mixed' for a precision given as a name or as FMM_PREC_*"""
    if isinstance(prec, str):
        return prec
    return "fp64" if int(prec) == 0 else "mixed"


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def gpu_fmm(fmm, ctx, w, p=None, theta=None, ncrit=None, precision=None, outputs=None, method=None, reps=1):
    """Returns (phi, E, tree) from the GPU path for workload w."""
    p = w.p if p is None else p
    theta = w.theta if theta is None else theta
    ncrit = w.ncrit if ncrit is None else ncrit
    precision = fmm.FMM_PREC_FP64 if precision is None else precision
    outputs = (fmm.FMM_POT | fmm.FMM_FIELD) if outputs is None else outputs
    method = fmm.FMM_METHOD_FMM if method is None else method
    pos = to_dev(w.pos)
    mom = to_dev(w.moments)
    t = fmm.Tree(ctx, pos, ncrit, theta, method)
    out = []
    for _ in range(reps):
        t.upward(w.order, mom, p, precision)
        phi, E = t.evaluate(outputs)
        torch.cuda.synchronize()
        out.append((None if phi is None else phi.cpu().numpy(), None if E is None else E.cpu().numpy()))
    if reps == 1:
        return out[0][0], out[0][1], t
    return out, t


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt((b * b).sum())
    return float(np.sqrt(((a - b) ** 2).sum()) / (den if den > 0 else 1.0))


def per_target(a, b, floor=1e-3):
    """largest over targets of |a_i - b_i| / max(|b_i|, floor * rms |b|)"""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    k = b.shape[0] if b.ndim else 1
    a = a.reshape(k, -1)
    b = b.reshape(k, -1)
    num = np.sqrt(((a - b) ** 2).sum(axis=1))
    mag = np.sqrt((b * b).sum(axis=1))
    rms = float(np.sqrt((mag * mag).mean())) if k else 0.0
    den = np.maximum(mag, floor * rms)
    if rms == 0.0:
        return float(num.max()) if k else 0.0
    return float((num / den).max())


def within(a, b, prec, label="", tol=None, floor=FIELD_FLOOR):
    """pooled and per-target errors of a against the reference b, printed;
    True when both are below the tolerances of the precision (or `tol`, a
    (pooled, per-target) pair); `floor`: PHI_FLOOR for potentials"""
    l2_tol, pt_tol = TOL[prec_name(prec)] if tol is None else tol
    e, m = rel_l2(a, b), per_target(a, b, floor)
    print(f"   {label}: rel L2 {e:.2e} (< {l2_tol:.0e}), max per target {m:.2e} (< {pt_tol:.0e})", flush=True)
    return e < l2_tol and m < pt_tol
