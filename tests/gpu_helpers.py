"""Shared helpers of the GPU parity tests: run the C-ABI library on seeded
inputs and compare with the oracle."""
import numpy as np
import torch


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
