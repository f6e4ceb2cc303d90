"""Serving: requests admitted by HBM footprint into resident slots, advanced
together in batched rounds, results moved to the host when done.

Each request's result (bonds, states, adjacency, positions, counters) must
equal the same replica run alone, whatever the mix it ran in; admission
must never exceed the budget; a request larger than the budget is refused."""
import threading
import time

import numpy as np
import pytest

from gpu_util import say
from paper_1409_7498_amd import workload

pytestmark = pytest.mark.gpu


def _reqs(n_req, seed, nmin=500, nmax=30000, steps_max=150):
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_req):
        N = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        kind = "step" if rng.random() < 0.5 else "chain"
        p = float(rng.uniform(0.001, 0.3))
        out.append((dict(n=N, L=workload.box_for(N), B=4 if kind == "step" else 2,
                         rule=workload.rule_for(kind, workload.RC, p), seed=int(seed * 1000 + r),
                         kind=kind, gen_seed=int(seed * 7 + r), sigma0=0.1, log_cap=4 * N),
                    int(rng.integers(1, steps_max))))
    return out


def _alone(B, d, steps, sigma):
    s = B.System(d["n"], d["L"], d["B"], d["rule"], d["seed"], log_cap=d["log_cap"])
    s.generate(d["kind"], d["gen_seed"], d["sigma0"])
    s.run(1, steps, sigma)
    out = (s.read(), s.bonds(), s.stats())
    s.close()
    return out


def test_served_results_equal_alone():
    """Staggered arrivals, a budget that holds a few replicas at a time and
    slots for four: every result equals the replica run alone."""
    from paper_1409_7498_amd import binding as B
    reqs = _reqs(14, 11)
    fps = [B.footprint(d, n) for d, n in reqs]
    budget = int(2.5 * max(fps))
    srv = B.Server(budget, 4)
    say("server budget", budget, "footprints", fps)
    used_max = [0]
    stop = [False]

    def watch():
        while not stop[0]:
            used_max[0] = max(used_max[0], srv.info()["used"])
            time.sleep(0.0005)

    th = threading.Thread(target=watch)
    th.start()
    tickets = []
    for k, (d, n) in enumerate(reqs):
        tickets.append(srv.submit(d, n, 0.05))
        time.sleep(0.002 * (k % 3))
    for t in tickets:
        st, code, lat = srv.wait(t, 120.0)
        assert st == B.Server.DONE, (t, st, code)
    stop[0] = True
    th.join()
    info = srv.info()
    say("server info", info, "max used", used_max[0])
    assert info["done"] == len(reqs) and info["failed"] == 0
    assert used_max[0] <= budget
    for t, (d, n) in zip(tickets, reqs):
        out, log, st = srv.read(t), srv.bonds(t), srv.stats(t)
        ref = _alone(B, d, n, 0.05)
        assert np.array_equal(log, ref[1]), t
        for k in ("x", "y", "z", "state", "adj"):
            assert np.array_equal(out[k], ref[0][k]), (t, k)
        assert st == ref[2], t
        srv.release(t)
    srv.close()


def test_same_result_alone_and_in_mix():
    """One request served alone and then inside a busy mix: identical."""
    from paper_1409_7498_amd import binding as B
    probe = _reqs(1, 23, nmin=5000, nmax=5000)[0]
    srv = B.Server(1 << 34, 8)
    t0 = srv.submit(probe[0], probe[1], 0.05)
    assert srv.wait(t0, 120.0)[0] == B.Server.DONE
    alone = (srv.read(t0), srv.bonds(t0), srv.stats(t0))
    mix = _reqs(10, 24)
    ts = [srv.submit(d, n, 0.05) for d, n in mix[:5]]
    t1 = srv.submit(probe[0], probe[1], 0.05)
    ts += [srv.submit(d, n, 0.05) for d, n in mix[5:]]
    assert srv.wait(t1, 120.0)[0] == B.Server.DONE
    for t in ts:
        assert srv.wait(t, 120.0)[0] == B.Server.DONE
    assert np.array_equal(srv.bonds(t1), alone[1])
    assert np.array_equal(srv.read(t1)["state"], alone[0]["state"])
    assert srv.stats(t1) == alone[2]
    srv.close()


def test_admission_refuses_oversize_and_reports():
    from paper_1409_7498_amd import binding as B
    d, n = _reqs(1, 31, nmin=20000, nmax=20000)[0]
    fp = B.footprint(d, n)
    srv = B.Server(fp - 1, 2)
    with pytest.raises(B.PrError) as e:
        srv.submit(d, n, 0.05)
    assert e.value.code == B.PR_EBUSY
    bad = dict(d, L=1.0)
    with pytest.raises(B.PrError) as e:
        srv.submit(bad, n, 0.05)
    assert e.value.code == B.PR_EINVAL
    with pytest.raises(B.PrError) as e:
        srv.wait(12345)
    assert e.value.code == B.PR_ENOTFOUND
    srv.close()


def test_cancel_queued_running_and_finished():
    """One slot: the first request runs while the others queue.  Cancelling a
    queued request fails it at once; cancelling the running one retires it at
    the end of its round; a finished request cannot be cancelled; the rest
    still equal their runs alone."""
    from paper_1409_7498_amd import binding as B
    reqs = _reqs(4, 31, nmin=20000, nmax=30000, steps_max=3)
    srv = B.Server(1 << 34, 1)
    long_req = dict(reqs[0][0])
    t_long = srv.submit(long_req, 3000, 0.05)
    others = [srv.submit(d, 40, 0.05) for d, _ in reqs[1:]]
    srv.cancel(others[0])
    st, code, _ = srv.poll(others[0])
    assert (st, code) == (3, B.PR_ECANCELED)
    t0 = time.time()
    while srv.poll(t_long)[0] == 0 and time.time() - t0 < 60:
        time.sleep(0.001)
    assert srv.poll(t_long)[0] == 1
    srv.cancel(t_long)
    st, code, _ = srv.wait(t_long, 60.0)
    assert (st, code) == (3, B.PR_ECANCELED)
    with pytest.raises(B.PrError) as e:
        srv.bonds(t_long)
    assert e.value.code == B.PR_ECANCELED
    for t in others[1:]:
        assert srv.wait(t, 120.0)[0] == 2
    with pytest.raises(B.PrError) as e:
        srv.cancel(others[1])
    assert e.value.code == B.PR_EBUSY
    with pytest.raises(B.PrError) as e:
        srv.cancel(12345678)
    assert e.value.code == B.PR_ENOTFOUND
    for (d, _), t in zip(reqs[2:], others[1:]):
        want = _alone(B, d, 40, 0.05)
        assert np.array_equal(srv.bonds(t), want[1])
        assert srv.stats(t) == want[2]
    info = srv.info()
    say("cancel: done", info["done"], "failed", info["failed"], "used", info["used"])
    assert info["failed"] == 2 and info["used"] == 0
    srv.close()
