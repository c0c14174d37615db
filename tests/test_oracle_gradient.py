"""Pins of the oracle's field gradient G_ij = d_i E_j = -d_i d_j phi
(Section 2: the derivative of order k = e_i + e_j of the local expansion;
the pair closed forms are the second derivatives of the sources' potentials).

Each check pins the gradient to something other than its own formula:
- central finite differences of the oracle's *field* (pair closed forms,
  the L2P field of Eq. 10, the direct sum with the target particle moved);
- the Laplace equation: phi is harmonic away from the sources, so
  trace(G) = 0 for every source order, traceless or not;
- the textbook charge gradient q (delta r^2 - 3 r r) / r^5;
- convergence of the FMM gradient to the direct one as p grows;
- exact superposition over the orders of a mixed system.
"""
import numpy as np
import pytest

import oracle

IJ = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def fd_of_field(field_at, x, h):
    """G_ij = d_i E_j by central differences of a field function."""
    G = np.zeros(6)
    for k, (i, j) in enumerate(IJ):
        e = np.zeros(3)
        e[i] = h
        G[k] = (field_at(x + e)[j] - field_at(x - e)[j]) / (2 * h)
    return G


MOMS = {0: np.array([1.7]), 1: np.array([0.4, -1.1, 0.8]),
        2: np.array([0.9, -0.3, 0.5, -0.2, 0.7, 0.6])}   # trace 1.3: not traceless on purpose


@pytest.mark.parametrize("order", [0, 1, 2])
def test_pair_gradient_is_derivative_of_pair_field(order):
    rng = np.random.default_rng(order)
    for _ in range(20):
        r = rng.uniform(-2, 2, 3)
        h = 1e-4 * np.linalg.norm(r)
        G = oracle.p2p_pair_grad(order, r, MOMS[order])
        Gfd = fd_of_field(lambda y: oracle.p2p_pair(order, y, MOMS[order])[1], r, h)
        assert np.abs(G - Gfd).max() <= 1e-6 * np.abs(G).max()


@pytest.mark.parametrize("order", [0, 1, 2])
def test_pair_gradient_traceless(order):
    rng = np.random.default_rng(10 + order)
    for _ in range(20):
        G = oracle.p2p_pair_grad(order, rng.uniform(-2, 2, 3), MOMS[order])
        assert abs(G[0] + G[3] + G[5]) <= 1e-12 * np.abs(G).max()


def test_charge_gradient_textbook():
    r = np.array([0.3, -0.7, 1.1])
    q = 2.5
    rn = np.linalg.norm(r)
    G = oracle.p2p_pair_grad(0, r, np.array([q]))
    want = [q * ((i == j) * rn * rn - 3 * r[i] * r[j]) / rn ** 5 for i, j in IJ]
    assert np.allclose(G, want, rtol=1e-14, atol=0)


def test_mixed_pair_is_sum_of_parts():
    r = np.array([0.5, 0.25, -0.75])
    mom = np.concatenate([MOMS[0], MOMS[1], MOMS[2]])
    G = oracle.p2p_pair_grad(oracle.mixed(7), r, mom)
    parts = sum(oracle.p2p_pair_grad(k, r, MOMS[k]) for k in range(3))
    assert np.allclose(G, parts, rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("p,s", [(4, 0), (6, 1), (10, 2), (3, 1)])
def test_l2p_gradient_is_derivative_of_l2p_field(p, s):
    rng = np.random.default_rng(p + s)
    L = rng.standard_normal(oracle.nterms(p - s))
    z = rng.uniform(-1, 1, 3)
    for _ in range(5):
        x = z + rng.uniform(-0.5, 0.5, 3)
        G = oracle.l2p_grad(p, s, z, L, x)
        Gfd = fd_of_field(lambda y: oracle.l2p(p, s, z, L, y)[1], x, 1e-4)
        assert np.abs(G - Gfd).max() <= 1e-7 * max(1.0, np.abs(G).max())


def test_l2p_gradient_vanishes_below_order_two():
    """p - s < 2: the truncated expansion is at most linear, so its second
    derivatives are zero (a finite difference of it gives the same)."""
    L = np.array([0.3, 1.0, -2.0, 0.5])
    x = np.array([0.1, -0.2, 0.3])
    assert np.all(oracle.l2p_grad(2, 1, np.zeros(3), L, x) == 0.0)
    Gfd = fd_of_field(lambda y: oracle.l2p(2, 1, np.zeros(3), L, y)[1], x, 1e-3)
    assert np.abs(Gfd).max() < 1e-9


@pytest.mark.parametrize("order", [0, 1, 2])
def test_direct_gradient_is_derivative_of_direct_field(order):
    rng = np.random.default_rng(50 + order)
    n = 300
    pos = rng.random((n, 3))
    mom = rng.standard_normal((n, [1, 3, 6][order]))
    tg = np.array([3, 77, 150, 299])
    G = oracle.direct_grad(pos, order, mom, targets=tg)
    h = 1e-5
    for k, i in enumerate(tg):
        def field_at(y, i=i):
            p2 = pos.copy()
            p2[i] = y
            return oracle.direct(p2, order, mom, targets=np.array([i]))[1][0]
        Gfd = fd_of_field(field_at, pos[i].copy(), h)
        assert np.abs(G[k] - Gfd).max() <= 1e-5 * np.abs(G[k]).max()
        assert abs(G[k, 0] + G[k, 3] + G[k, 5]) <= 1e-10 * np.abs(G[k]).max()


@pytest.mark.parametrize("order", [0, 1, 2])
def test_fmm_gradient_converges_to_direct(order):
    rng = np.random.default_rng(70 + order)
    n = 2000
    pos = rng.random((n, 3))
    mom = rng.standard_normal((n, [1, 3, 6][order]))
    Gd = oracle.direct_grad(pos, order, mom)
    t = oracle.Tree(pos, 16, 0.5)
    errs = []
    for p in (order + 2, order + 4, order + 6, 10):
        _, _, G = t.fmm(order, mom, p, want_grad=True)
        errs.append(oracle.rel_l2(G, Gd))
    # the truncation error falls with p (and is not zero to begin with)
    assert errs[-1] < 1e-4 and errs[-1] < errs[0] / 3 and errs[0] > 1e-8, errs
    assert all(b <= a * 1.05 for a, b in zip(errs, errs[1:])), errs


def test_fmm_gradient_mixed_superposes():
    """A charge + dipole + quadrupole system: its gradient is the sum of its
    parts' on the same tree and truncation (the charge part alone has the
    same lowest order, so it runs as a plain charge system)."""
    rng = np.random.default_rng(91)
    n = 1500
    pos = rng.random((n, 3))
    m0, m1, m2 = rng.standard_normal((n, 1)), rng.standard_normal((n, 3)), rng.standard_normal((n, 6))
    z1, z3, z6 = np.zeros((n, 1)), np.zeros((n, 3)), np.zeros((n, 6))
    t = oracle.Tree(pos, 24, 0.5)
    p, code = 6, oracle.mixed(7)
    G = t.fmm(code, np.hstack([m0, m1, m2]), p, want_grad=True)[2]
    parts = (t.fmm(0, m0, p, want_grad=True)[2] + t.fmm(code, np.hstack([z1, m1, z6]), p, want_grad=True)[2]
             + t.fmm(code, np.hstack([z1, z3, m2]), p, want_grad=True)[2])
    assert np.abs(G - parts).max() <= 1e-12 * np.abs(G).max()


@pytest.mark.parametrize("p,s", [(4, 0), (6, 1), (8, 2), (1, 1)])
def test_m2p_gradient_is_derivative_of_m2p_field(p, s):
    """Barnes-Hut: the gradient of the multipole's own field (finite
    differences of the oracle's M2P field)."""
    rng = np.random.default_rng(200 + p + s)
    M = rng.standard_normal(oracle.nterms(p))
    M[:oracle.nterms(s - 1)] = 0.0
    zA = rng.uniform(-0.2, 0.2, 3)
    for _ in range(4):
        x = zA + rng.uniform(1.5, 2.5, 3) * rng.choice([-1, 1], 3)
        G = oracle.m2p_grad(p, s, zA, M, x)
        Gfd = fd_of_field(lambda y: oracle.m2p(p, s, zA, M, y)[1], x, 1e-5)
        assert np.abs(G - Gfd).max() <= 1e-6 * np.abs(G).max()
        assert abs(G[0] + G[3] + G[5]) <= 1e-12 * np.abs(G).max()


@pytest.mark.parametrize("order", [0, 1, 2])
def test_bh_gradient_converges_to_direct(order):
    rng = np.random.default_rng(300 + order)
    n = 1500
    pos = rng.random((n, 3))
    mom = rng.standard_normal((n, [1, 3, 6][order]))
    Gd = oracle.direct_grad(pos, order, mom)
    t = oracle.Tree(pos, 16)
    errs = [oracle.rel_l2(t.bh(order, mom, p, 0.5, want_grad=True)[2], Gd) for p in (max(order, 1), order + 3, 8)]
    # the far part shrinks with p (slowly where the near field dominates)
    assert errs[2] < errs[1] < errs[0] and errs[-1] < 2e-3, errs
    # a tiny opening angle accepts nothing: the direct sum itself
    G0 = t.bh(order, mom, 4, 1e-6, want_grad=True)[2]
    assert oracle.rel_l2(G0, Gd) < 1e-13
