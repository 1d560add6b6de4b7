"""Candidate enumeration on the device (fpt_enumerate, through the C ABI)
against the enumeration oracle: bit-exact on every candidate of small
specs (whole range and ragged windows), on all 6,270,016 candidates of the
order <= 2 canyon workload (against the host generator, which the oracle's
pins tie to the definition), and on sampled ranks of the order 1..6 canyon
candidate set (5.9e16 candidates) unranked by the oracle one by one."""
import numpy as np
import pytest

from oracle import candidates as cand
from paper_2510_16172_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2510_16172_amd import fpt
    s = fpt.Solver(0)
    yield s
    s.close()


def _pairs(P, seed=0):
    import torch
    rng = np.random.default_rng(seed)
    ps = rng.integers(0, 1000, P).astype(np.int32)
    pd = rng.integers(0, 1000, P).astype(np.int32)
    return ps, pd, torch.from_numpy(ps).cuda(), torch.from_numpy(pd).cuda()


def _host(out):
    import torch
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _expect(c, ps, pd, n_max):
    N = len(c)
    src = np.array([ps[p] for p, _ in c], np.int32).reshape(N)
    dst = np.array([pd[p] for p, _ in c], np.int32).reshape(N)
    order = np.array([len(s) for _, s in c], np.uint8).reshape(N)
    ids = np.full((n_max, N), -1, np.int32)
    for i, (_, s) in enumerate(c):
        ids[: len(s), i] = s
    return {"src": src, "dst": dst, "order": order, "ids": ids}


def _assert_equal(got, want):
    for k in ("src", "dst", "order", "ids"):
        np.testing.assert_array_equal(got[k], want[k], err_msg=k)


@pytest.mark.parametrize("P,K,lo,hi,nr,n_max",
                         [(3, 4, 1, 3, True, 3), (2, 3, 2, 4, False, 6), (1, 1, 1, 3, True, 3),
                          (2, 2, 1, 6, True, 6), (5, 7, 1, 2, True, 4)])
def test_small_specs_match_oracle(solver, P, K, lo, hi, nr, n_max):
    ps, pd, tps, tpd = _pairs(P, seed=P * 100 + K)
    c = cand.candidates(P, K, lo, hi, nr)
    total = len(c)
    from paper_2510_16172_amd import fpt
    assert fpt.enum_count(P, K, lo, hi, nr) == total
    got = _host(solver.enumerate(tps, tpd, K, lo, hi, nr, n_max=n_max))
    _assert_equal(got, _expect(c, ps, pd, n_max))
    # ragged windows, including an empty one and the last candidate alone
    rng = np.random.default_rng(total)
    wins = [(0, 0), (total - 1, 1), (total // 3, total - total // 3)]
    wins += [(int(a), int(rng.integers(0, total - a + 1))) for a in rng.integers(0, total, 4)]
    for r0, cnt in wins:
        got = _host(solver.enumerate(tps, tpd, K, lo, hi, nr, rank0=r0, count=cnt,
                                     n_max=n_max))
        _assert_equal(got, _expect(c[r0:r0 + cnt], ps, pd, n_max))


def test_errors(solver):
    from paper_2510_16172_amd import fpt
    _, _, tps, tpd = _pairs(3)
    total = fpt.enum_count(3, 4, 1, 2)
    with pytest.raises(fpt.FptError):
        solver.enumerate(tps, tpd, 4, 1, 2, rank0=total - 5, count=6)
    with pytest.raises(fpt.FptError):
        solver.enumerate(tps, tpd, 4, 1, 2, rank0=-1, count=1)
    with pytest.raises(fpt.FptError):
        solver.enumerate(tps, tpd, 4, 1, 3, n_max=2, count=1)


def test_order2_canyon_all_candidates(solver):
    """All 6,270,016 candidates of the order <= 2 canyon workload in one
    launch, equal to the host generator's arrays."""
    import torch
    sc = scenes.canyon_scene()
    b = scenes.canyon_all_paths(sc, n_max=2)
    P = sc.meta["n_pairs"]
    tps = torch.arange(0, 2 * P, 2, dtype=torch.int32, device="cuda")
    tpd = tps + 1
    got = _host(solver.enumerate(tps, tpd, sc.K, 1, 2))
    _assert_equal(got, {"src": b.src, "dst": b.dst, "order": b.order, "ids": b.ids})


def test_order6_canyon_sampled_ranks(solver):
    """Chunks of the order 1..6 canyon candidate set (64 pairs, 313 objects,
    5.9e16 candidates): first, middle and last 2^17 ranks; 300 sampled
    positions per chunk unranked by the oracle; every candidate of the
    chunks checked for range, no immediate repeat and increasing rank."""
    import torch
    from paper_2510_16172_amd import fpt
    P, K = 64, 313
    ps = (3 * np.arange(P) + 1).astype(np.int32)  # increasing: src orders the pairs
    pd = ps + 1
    tps, tpd = torch.from_numpy(ps).cuda(), torch.from_numpy(pd).cuda()
    total = fpt.enum_count(P, K, 1, 6)
    assert total == cand.total(P, K, 1, 6)
    cnt = 1 << 17
    rng = np.random.default_rng(66)
    for r0 in (0, int(rng.integers(0, total - cnt)), total - cnt):
        got = _host(solver.enumerate(tps, tpd, K, 1, 6, rank0=r0, count=cnt))
        for i in np.sort(rng.choice(cnt, 300, replace=False)):
            p, s = cand.unrank(r0 + int(i), P, K, 1, 6)
            assert got["src"][i] == ps[p] and got["dst"][i] == pd[p]
            assert got["order"][i] == len(s)
            assert tuple(got["ids"][: len(s), i]) == s and np.all(got["ids"][len(s):, i] == -1)
        ids, order = got["ids"].astype(np.int64), got["order"].astype(np.int64)
        j = np.arange(6)[:, None]
        act = j < order[None, :]
        assert np.all(np.where(act, (ids >= 0) & (ids < K), ids == -1))
        assert np.all(~(act[1:] & (ids[1:] == ids[:-1])))
        # strictly increasing (order, pair, sequence) from one rank to the next
        key = np.concatenate([order[None], got["src"][None].astype(np.int64), ids], axis=0)
        prev, cur = key[:, :-1], key[:, 1:]
        diff = prev != cur
        assert np.all(diff.any(axis=0))
        first = np.argmax(diff, axis=0)[None]
        assert np.all(np.take_along_axis(prev, first, 0) < np.take_along_axis(cur, first, 0))


def test_enumerate_then_solve_equals_host_batch(solver):
    """A window of device-enumerated candidates solves to the same bits as
    the same candidates built on the host."""
    import torch
    from paper_2510_16172_amd import fpt
    sc = scenes.canyon_scene()
    b = scenes.canyon_all_paths(sc, n_max=2)
    r0, cnt = 1_000_003, 200_001
    P = sc.meta["n_pairs"]
    tps = torch.arange(0, 2 * P, 2, dtype=torch.int32, device="cuda")
    e = solver.enumerate(tps, tps + 1, sc.K, 1, 2, rank0=r0, count=cnt)
    obj = torch.from_numpy(sc.obj).cuda()
    pts = torch.from_numpy(sc.pts).cuda()
    dbe = fpt.DeviceBatch.from_tensors(obj, pts, e["src"], e["dst"], e["ids"], e["order"], S=b.S)
    dbh = fpt.DeviceBatch(b.subset(np.arange(r0, r0 + cnt)))
    opts = fpt.Opts(scale=b.S, iters=16)
    oe = {k: v.cpu().numpy() for k, v in solver.solve(dbe, opts).items()}
    oh = {k: v.cpu().numpy() for k, v in solver.solve(dbh, opts).items()}
    for k in oe:
        np.testing.assert_array_equal(oe[k], oh[k], err_msg=k)
