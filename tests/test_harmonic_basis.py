"""The harmonic (reduced) M2L basis, checked on the CPU against the oracle.

The GPU folds each multipole onto its components with m_z <= 1, contracts
only those against the derivative tensor, produces the local components with
n_z <= 1, and rebuilds the others.  All of it rests on D being harmonic
(the derivatives of 1/r), so the identities are checked with the oracle's
own M2L and derivative tensor, not with anything the GPU path computes:

- folding the multipole leaves the oracle's M2L unchanged (every component);
- the oracle's locals satisfy the rebuild rule exactly (up to rounding);
- the generated kernels' term lists (components, derivative indices,
  truncation) reproduce the oracle's locals from the folded multipole;
- the derivative tensor itself is traceless (the property the rest needs).
The folding and rebuild formulas are written out here again from the
identity D_{k+2j e_z} = (-1)^j sum_i C(j,i) D_{k+2i e_x+2(j-i) e_y}.
"""
import os
import sys
from math import comb

import numpy as np
import pytest

import oracle

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", "paper_2005_12351_amd", "csrc"))
import gen_m2l  # noqa: E402

sys.path.pop(0)


def mis(p):
    return [oracle.multi_index(i) for i in range(oracle.nterms(p))]


def fold(p, s, M):
    """Multipole (all components up to order p in storage order, those below
    order s zero, the layout the oracle's M2L takes) folded onto the
    components with m_z <= 1; zeros at m_z >= 2."""
    out = np.zeros_like(M)
    for j, (a, b, r) in enumerate(mis(p)):
        if r > 1 or a + b + r < s:
            continue
        acc = 0.0
        for jj in range((a + b) // 2 + 1):
            for i in range(jj + 1):
                ax, by = a - 2 * i, b - 2 * (jj - i)
                if ax < 0 or by < 0:
                    continue
                acc += (-1) ** jj * comb(jj, i) * M[oracle.index(ax, by, r + 2 * jj)]
        out[j] = acc
    return out


def rebuild(q, L):
    """Locals with n_z >= 2 from those with n_z <= 1."""
    out = L.copy()
    for k, (a, b, c) in enumerate(mis(q)):
        if c <= 1:
            continue
        j, r = divmod(c, 2)
        out[k] = (-1) ** j * sum(comb(j, i) * L[oracle.index(a + 2 * i, b + 2 * (j - i), r)] for i in range(j + 1))
    return out


CASES = [(4, 0), (6, 1), (8, 1), (10, 1), (10, 2), (5, 2)]


def _pair(seed, p, s):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal(oracle.nterms(p))
    M[:oracle.nterms(s - 1)] = 0.0
    zA = rng.uniform(-0.5, 0.5, 3)
    zB = zA + rng.uniform(2.0, 3.0, 3) * rng.choice([-1, 1], 3)
    return M, zA, zB


@pytest.mark.parametrize("p,s", CASES)
def test_dtensor_is_traceless(p, s):
    D = oracle.dtensor(p, np.array([0.7, -1.3, 0.4]))
    for k, (a, b, c) in enumerate(mis(p - 2)):
        tr = D[oracle.index(a + 2, b, c)] + D[oracle.index(a, b + 2, c)] + D[oracle.index(a, b, c + 2)]
        scale = abs(D[oracle.index(a + 2, b, c)]) + abs(D[oracle.index(a, b, c + 2)])
        assert abs(tr) <= 1e-12 * scale


@pytest.mark.parametrize("p,s", CASES)
def test_folded_multipole_gives_same_locals(p, s):
    M, zA, zB = _pair(p * 10 + s, p, s)
    L = oracle.m2l(p, s, zA, M, zB)
    Mf = fold(p, s, M)
    assert np.abs(Mf - M).max() > 1e-3          # the folding is not the identity
    Lf = oracle.m2l(p, s, zA, Mf, zB)
    assert np.abs(Lf - L).max() <= 1e-11 * np.abs(L).max()


@pytest.mark.parametrize("p,s", CASES)
def test_locals_obey_rebuild_rule(p, s):
    M, zA, zB = _pair(p * 10 + s + 1, p, s)
    L = oracle.m2l(p, s, zA, M, zB)
    kept = np.array([c <= 1 for (_, _, c) in mis(p - s)])
    Lr = rebuild(p - s, np.where(kept, L, np.nan))
    assert np.all(np.isfinite(Lr))
    assert np.abs(Lr - L).max() <= 1e-11 * np.abs(L).max()


@pytest.mark.parametrize("p,s", CASES)
def test_generated_term_lists(p, s):
    """The kernel's reduced rows: the components it keeps, their order in a
    row, and the multiply-adds (output n, input m, derivative index n+m)."""
    M, zA, zB = _pair(p * 10 + s + 2, p, s)
    L = oracle.m2l(p, s, zA, M, zB)
    D = oracle.dtensor(p, zB - zA)
    n0 = oracle.nterms(s - 1)
    Mf = fold(p, s, M)
    ns = gen_m2l.reduced(gen_m2l.orders(p - s))
    ms = gen_m2l.reduced(gen_m2l.orders(p)[n0:])
    assert len(ns) == (p - s + 1) ** 2 and len(ms) == (p + 1) ** 2 - s ** 2
    Mh = np.array([Mf[oracle.index(*m)] for m in ms])
    Lh = np.zeros(len(ns))
    for i, n in enumerate(ns):
        for j, m in enumerate(ms):
            if sum(n) + sum(m) <= p:
                Lh[i] += Mh[j] * D[gen_m2l.idx((n[0] + m[0], n[1] + m[1], n[2] + m[2]))]
    full = np.zeros(oracle.nterms(p - s))
    for i, n in enumerate(ns):
        full[oracle.index(*n)] = Lh[i]
    Lr = rebuild(p - s, full)
    assert np.abs(Lr - L).max() <= 1e-11 * np.abs(L).max()
    # the per-block counts the host's cost model uses
    _, meta = gen_m2l.gen_kernel(p, s, True, None, True)
    assert sum(meta["bfma"]) == sum(1 for n in ns for m in ms if sum(n) + sum(m) <= p)


def test_multiply_add_counts():
    """Multiply-adds per M2L list entry: full and harmonic basis."""
    def count(p, s, harm):
        ns = gen_m2l.orders(p - s)
        ms = gen_m2l.orders(p)[oracle.nterms(s - 1):]
        if harm:
            ns, ms = gen_m2l.reduced(ns), gen_m2l.reduced(ms)
        return sum(1 for n in ns for m in ms if sum(n) + sum(m) <= p)
    assert count(8, 1, False) == 2838 and count(8, 1, True) == 1284
    assert count(10, 2, False) == 7062 and count(10, 2, True) == 2505
    # closed form of the harmonic count: sum_l (2l+1) ((p-l+1)^2 - s^2)
    for p, s in CASES:
        assert count(p, s, True) == sum((2 * l + 1) * ((p - l + 1) ** 2 - s ** 2) for l in range(p - s + 1))
