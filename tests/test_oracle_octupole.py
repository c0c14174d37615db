"""Pins of the oracle's octupole sources (source order 3; Section 2: sources
of any order 2^n enter through their source tensor, Eq. 5).  The octupole
moment is O_m = sum q x^m over a charge distribution (the ten components of
order 3 in the index order); the pins tie the closed forms and the source
tensor S_m = -O_m / m! to that definition: a cluster of point charges whose
lower moments vanish tends to the point octupole as it shrinks."""
import math

import numpy as np
import pytest

from paper_2005_12351_amd import workloads as W

C4 = np.array([-1.0, 3.0, -3.0, 1.0])   # third difference: kills orders 0-2 (and 4, about the midpoint)


def _charges_for(O, a, rng):
    """40 charges with raw octupole O (any symmetric tensor), vanishing
    charge, dipole and quadrupole, as ten linear octupoles along random
    directions n: charges C4 w / (6 a^3) at (k - 3/2) a n"""
    dirs = rng.standard_normal((10, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    A = np.array([[d[0] ** c[0] * d[1] ** c[1] * d[2] ** c[2] for d in dirs] for c in W.OCT_INDEX])
    w = np.linalg.solve(A, O)
    pos = np.concatenate([np.outer(np.arange(4) - 1.5, d) * a for d in dirs])
    q = np.concatenate([C4 * wl / (6.0 * a ** 3) for wl in w])
    return pos, q


def _cluster_field(orc, pos, q, x):
    ph, E, G = 0.0, np.zeros(3), np.zeros(6)
    for xj, qj in zip(pos, q):
        p_, e_ = orc.p2p_pair(0, x - xj, [qj])
        ph += p_
        E += e_
        G += orc.p2p_pair_grad(0, x - xj, [qj])
    return ph, E, G


def test_raw_moments_of_the_cluster(orc):
    rng = np.random.default_rng(3)
    O = rng.standard_normal(10)
    pos, q = _charges_for(O, 0.01, rng)
    for K in range(3):
        for c in [(nx, ny, K - nx - ny) for nx in range(K, -1, -1) for ny in range(K - nx, -1, -1)]:
            assert abs(np.sum(q * np.prod(pos ** np.array(c), axis=1))) < 1e-9
    got = [np.sum(q * np.prod(pos ** np.array(c), axis=1)) for c in W.OCT_INDEX]
    assert np.allclose(got, O, rtol=1e-9, atol=1e-9)


def test_octupole_is_the_limit_of_point_charges(orc):
    """potential, field and field gradient of the shrinking cluster against
    the closed forms (general, not traceless, tensors): the error falls as
    a^2 (the cluster's fourth moment vanishes about its centre)"""
    rng = np.random.default_rng(5)
    for trial in range(4):
        O = rng.standard_normal(10)
        x = rng.standard_normal(3)
        x *= rng.uniform(0.8, 1.5) / np.linalg.norm(x)
        ph, E = orc.p2p_pair(3, x, O)
        G = orc.p2p_pair_grad(3, x, O)
        errs = []
        for a in (0.01, 0.005):
            pos, q = _charges_for(O, a, np.random.default_rng(100 + trial))
            cp, cE, cG = _cluster_field(orc, pos, q, x)
            errs.append(max(abs(cp - ph) / abs(ph), np.abs(cE - E).max() / np.abs(E).max(),
                            np.abs(cG - G).max() / np.abs(G).max()))
        assert errs[1] < errs[0] / 3.0 and errs[1] < 1e-3, errs


def test_octupole_closed_forms_match_the_derivative_tensor(orc):
    """order 1 and 2 derivatives from S_m D_{m+k} (source tensor and the
    recurrence for D) equal -E and -G of the closed forms, and E and G are
    the derivatives of phi and E (central differences)"""
    rng = np.random.default_rng(7)
    h = 1e-5
    for _ in range(10):
        O = rng.standard_normal(10)
        x = rng.standard_normal(3) + np.array([1.0, 0.0, 0.0])
        ph, E = orc.p2p_pair(3, x, O)
        G = orc.p2p_pair_grad(3, x, O)
        assert np.allclose(orc.pair_derivs(3, 1, x, O), -E, rtol=1e-12, atol=1e-13 * np.abs(E).max())
        assert np.allclose(orc.pair_derivs(3, 2, x, O), -G, rtol=1e-12, atol=1e-13 * np.abs(G).max())
        # phi from the derivative tensor: sum_m S_m D_m
        D = orc.dtensor(3, x)
        S = [-O[c] / np.prod([math.factorial(e) for e in W.OCT_INDEX[c]]) for c in range(10)]
        assert abs(sum(S[c] * D[orc.index(*W.OCT_INDEX[c])] for c in range(10)) - ph) <= 1e-13 * abs(ph) + 1e-15
        for l in range(3):
            e = np.zeros(3)
            e[l] = h
            fdE = -(orc.p2p_pair(3, x + e, O)[0] - orc.p2p_pair(3, x - e, O)[0]) / (2 * h)
            assert abs(fdE - E[l]) <= 1e-6 * np.abs(E).max()


def test_traceless_octupole_has_no_trace_terms(orc):
    """for a traceless tensor phi = 5/2 O(r,r,r) / r^7 exactly"""
    rng = np.random.default_rng(9)
    O = W.random_moments(rng, 3, 1)[0]
    T = W.octupole_full(O)[0]
    x = np.array([0.3, -0.7, 0.5])
    r = np.linalg.norm(x)
    assert np.isclose(orc.p2p_pair(3, x, O)[0], 2.5 * np.einsum("ijk,i,j,k->", T, x, x, x) / r ** 7, rtol=1e-13)


def test_fmm_octupoles_converge_to_direct(orc):
    w = W.small_random(11, 2000, 3, "plummer")
    d_ph, d_E = orc.direct(w.pos, 3, w.moments)
    t = orc.Tree(w.pos, 32, 0.5)
    errs = []
    for p in (4, 6, 8, 10):
        ph, E = t.fmm(3, w.moments, p)[:2]
        errs.append((orc.rel_l2(ph, d_ph), orc.rel_l2(E, d_E)))
    assert all(b[1] < a[1] for a, b in zip(errs, errs[1:])), errs
    assert errs[-1][0] < 1e-3 and errs[-1][1] < 1e-3, errs
    # p = s: no far field; a single leaf: the direct sum itself
    t1 = orc.Tree(w.pos[:40], 64, 0.5)
    ph, E = t1.fmm(3, w.moments[:40], 4)[:2]
    d_ph, d_E = orc.direct(w.pos[:40], 3, w.moments[:40])
    assert orc.rel_l2(ph, d_ph) < 1e-14 and orc.rel_l2(E, d_E) < 1e-14


def test_bh_octupoles_converge_to_direct(orc):
    w = W.small_random(13, 1500, 3, "uniform")
    d_ph, d_E = orc.direct(w.pos, 3, w.moments)
    t = orc.Tree(w.pos, 16)
    errs = [orc.rel_l2(t.bh(3, w.moments, p, 0.5)[1], d_E) for p in (3, 6, 9)]
    assert errs[2] < errs[1] < errs[0] and errs[-1] < 2e-3, errs


def test_mixed_with_octupoles_superposes(orc):
    """charges + octupoles (mask 9) and all four orders (mask 15): each the
    sum of its single-order systems"""
    w = W.small_mixed(15, 800, 15, "plummer")
    m = w.moments
    parts = {0: m[:, :1], 1: m[:, 1:4], 2: m[:, 4:10], 3: m[:, 10:20]}
    t = orc.Tree(w.pos, 16, 0.5)
    p = 7
    ph, E = t.fmm(orc.mixed(15), m, p)[:2]
    # the expansions of the whole system start at order 0; each part alone
    # starts at its own order, so compare against the parts in one system
    # with the others zeroed
    acc_ph, acc_E = 0.0, 0.0
    for k in range(4):
        z = np.zeros_like(m)
        lo = {0: 0, 1: 1, 2: 4, 3: 10}[k]
        z[:, lo:lo + parts[k].shape[1]] = parts[k]
        a, b = t.fmm(orc.mixed(15), z, p)[:2]
        acc_ph = acc_ph + a
        acc_E = acc_E + b
    assert orc.rel_l2(ph, acc_ph) < 1e-12 and orc.rel_l2(E, acc_E) < 1e-12
    # charges + octupoles against the direct sum
    m9 = np.hstack([parts[0], parts[3]])
    ph9, E9 = t.fmm(orc.mixed(9), m9, 8)[:2]
    dph, dE = orc.direct(w.pos, orc.mixed(9), m9)
    assert orc.rel_l2(E9, dE) < 2e-3
