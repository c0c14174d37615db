"""The M2L schedule built on the device against the one the host threads
build: the same tiles, class ids, per-lane sources and class geometries,
entry for entry, and the same FMM results bit for bit.  Independently of
both builders, the schedule must cover every M2L pair of the exported lists
exactly once, at the class whose geometry is that pair's exact
((z_B - z_A) / r_B, r_A / r_B) (Section 3.3, Eq. 8)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2005_12351_amd import fmm  # noqa: E402
from paper_2005_12351_amd import workloads as W  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctxs():
    dev = fmm.Context(0)
    dev.set_m2l_schedule(fmm.FMM_SCHEDULE_DEVICE)
    host = fmm.Context(0)
    host.set_m2l_schedule(fmm.FMM_SCHEDULE_HOST)
    yield dev, host
    dev.close()
    host.close()


# (kind, n, ncrit, theta): uniform and clustered (cross-level pairs), a
# lattice, one particle per leaf, trees without any M2L pair, clustered
# trees whose tiles hold 2000-3000 distinct pair geometries
CASES = [("uniform", 20000, 32, 0.3), ("uniform", 20000, 64, 0.5), ("plummer", 30000, 16, 0.6),
         ("plummer", 8000, 1, 0.4), ("lattice", 4096, 64, 0.5), ("uniform", 777, 1, 0.4),
         ("uniform", 100, 64, 0.5), ("uniform", 1, 8, 0.5), ("uniform", 2, 1, 0.5),
         ("plummer", 12000, 16, 0.5), ("plummer", 9000, 1, 0.4)]


def _check_cover(sch, ex):
    """every (target, source) pair of the lists once, at its exact class"""
    nc = len(ex["level"])
    lvl, ix = ex["level"].astype(np.int64), ex["ix"].astype(np.int64)
    tc, uoff, ucls, usrc, geom = sch["tile_cell"], sch["tile_uoff"], sch["ucls"], sch["usrc"], sch["cls_geom"]
    ptr, src = ex["m2l_ptr"], ex["m2l_src"]
    targets = np.nonzero(ptr[1:] > ptr[:-1])[0]
    assert np.array_equal(np.sort(tc[tc >= 0]), targets)
    assert np.all(tc[len(targets):] == -1)
    ntl = len(uoff) - 1
    if ntl == 0:
        assert len(src) == 0 and len(ucls) == 0
        return
    tile = np.repeat(np.arange(ntl), np.diff(uoff))
    first = np.zeros(len(ucls), bool)
    first[uoff[:-1]] = True
    assert np.all(first | (np.diff(ucls, prepend=-1) > 0))   # ascending and distinct within a tile
    B = tc.reshape(ntl, 64)[tile]                              # (entries, 64) target of each lane
    rows = usrc.reshape(-1, 64)
    assert np.all(rows[B < 0] == nc)
    real = rows != nc
    A, Bv, c = rows[real].astype(np.int64), B[real].astype(np.int64), np.broadcast_to(ucls[:, None], rows.shape)[real]
    assert np.all(Bv >= 0)
    # the multiset of (target, source) pairs is the lists'
    got = np.sort(Bv * nc + A)
    want = np.sort(np.repeat(np.arange(nc), np.diff(ptr)) * nc + src)
    assert np.array_equal(got, want)
    # each pair sits at the class of its exact geometry
    lm = np.maximum(lvl[A], lvl[Bv])
    d = ((2 * ix[Bv] + 1) << (lm - lvl[Bv])[:, None]) - ((2 * ix[A] + 1) << (lm - lvl[A])[:, None])
    dl = lvl[Bv] - lvl[A]
    unit = np.ldexp(1.0, np.minimum(0, dl))
    exp = np.concatenate([d * unit[:, None], np.ldexp(1.0, dl)[:, None]], axis=1)
    assert np.array_equal(geom[c], exp)


@pytest.mark.parametrize("kind,n,ncrit,theta", CASES)
def test_device_schedule_matches_host(ctxs, kind, n, ncrit, theta):
    _say(f"[schedule] {kind} n={n} ncrit={ncrit} theta={theta}")
    dev, host = ctxs
    w = W.small_random(900 + n, n, 1, kind, p=6)
    pos = torch.from_numpy(w.pos).cuda()
    td = fmm.Tree(dev, pos, ncrit, theta)
    th = fmm.Tree(host, pos, ncrit, theta)
    a, b = td.m2l_schedule(), th.m2l_schedule()
    assert a["where"] == fmm.FMM_SCHEDULE_DEVICE and b["where"] == fmm.FMM_SCHEDULE_HOST
    ia, ib = td.info(), th.info()
    for k in ("n_m2l", "n_classes", "n_tiles", "m2l_slots"):
        assert ia[k] == ib[k], k
    for k in ("tile_cell", "tile_uoff", "ucls", "usrc", "cls_geom"):
        assert a[k].shape == b[k].shape, k
        assert np.array_equal(a[k], b[k]), k
    _check_cover(a, td.export())
    # the same schedule gives the same results, bit for bit
    mom = torch.from_numpy(w.moments).cuda()
    outs = []
    for t in (td, th):
        t.upward(1, mom, 6, fmm.FMM_PREC_MIXED)
        phi, field = t.evaluate()
        torch.cuda.synchronize()
        outs.append((phi.cpu().numpy(), field.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    td.close()
    th.close()


def test_device_schedule_serving(ctxs):
    """a tree built, evaluated and rebuilt on the same context reuses the
    device path each time (no stale state between builds)"""
    dev, _ = ctxs
    rng = np.random.default_rng(7)
    for n in (5000, 300, 12000):
        _say(f"[schedule rebuild] n={n}")
        w = W.small_random(int(rng.integers(1 << 30)), n, 1, "plummer", p=5)
        pos = torch.from_numpy(w.pos).cuda()
        t = fmm.Tree(dev, pos, 16, 0.5)
        s = t.m2l_schedule()
        assert s["where"] == fmm.FMM_SCHEDULE_DEVICE
        _check_cover(s, t.export())
        t.close()


def test_schedule_auto():
    """the default takes the device for small and large trees alike, and
    gives the host's schedule"""
    auto = fmm.Context(0)
    host = fmm.Context(0)
    host.set_m2l_schedule(fmm.FMM_SCHEDULE_HOST)
    for n in (1000, 40000):
        w = W.small_random(77 + n, n, 1, "uniform")
        pos = torch.from_numpy(w.pos).cuda()
        ta, th = fmm.Tree(auto, pos, 64, 0.5), fmm.Tree(host, pos, 64, 0.5)
        a, b = ta.m2l_schedule(), th.m2l_schedule()
        _say(f"[schedule auto] n={n} n_m2l={ta.info()['n_m2l']} where={a['where']}")
        assert a["where"] == fmm.FMM_SCHEDULE_DEVICE
        for k in ("tile_cell", "tile_uoff", "ucls", "usrc", "cls_geom"):
            assert np.array_equal(a[k], b[k]), k
        ta.close()
        th.close()
    auto.close()
    host.close()


def test_schedule_setter_rejects(ctxs):
    dev, _ = ctxs
    with pytest.raises(fmm.FMMError):
        dev.set_m2l_schedule(3)
