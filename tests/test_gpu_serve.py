"""Request server on the GPU: solves admitted by footprint and overlapped on
several streams give the same results as the same solves run alone (bit for
bit: each solve has its own context and deterministic kernels), and match the
oracle.  Admission is exercised with an arena too small for all requests at
once."""
import numpy as np
import pytest

import synth
from tests._gpu import need_gpu, rel_err

pytestmark = pytest.mark.gpu


def _requests(count, seed, lo=10.0, hi=15.0):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(np.rint(2.0 ** rng.uniform(lo, hi)))
        model = "plummer" if rng.random() < 0.5 else "cube"
        x, _, m = (synth.plummer if model == "plummer" else synth.cold_cube)(n, seed * 1000 + k)
        if k % 2:
            m = synth.lognormal_masses(n, seed * 1000 + k + 500)
        R2 = synth.r2_for_neighbours(model, n, 64)
        pad = int(rng.integers(0, 300))
        xb = np.zeros((3, n + pad))
        xb[:, :n] = x
        out.append(dict(n=n, x=x, xb=xb, m=m.astype(np.float32), hybrid=int(k % 5 != 4),
                        theta=float(rng.uniform(0.4, 0.7)), eps=0.01 * (2.0 ** 20 / n) ** (1 / 3),
                        R2=R2, pot=(k % 3 == 0), G=(1.0, 2.5, 2.0 ** 20 / n)[k % 3]))
    return out


def _params(P, r):
    return P.default_params(G=r["G"], eps=r["eps"], theta=r["theta"], R1=r["R2"] / 2,
                            R2=r["R2"], hybrid=r["hybrid"], flags=P.F_POT if r["pot"] else 0)


def _collect(P, torch, srv, reqs, ids, keep, limit_s=60.0):
    """Polls until every id has finished; copies results out, releases."""
    import time
    got = {}
    t_end = time.monotonic() + limit_s
    while len(got) < len(ids):
        assert time.monotonic() < t_end, "requests did not finish: %s" % srv.stats()
        for rid in srv.poll():
            inf, a_s, a_h, ngb, pot = srv.result(rid)
            got[rid] = (inf, *(None if t is None else t.clone() for t in (a_s, a_h, ngb, pot)))
            # the copies must be done before the block can be reused
            torch.cuda.current_stream().synchronize()
            if not keep:
                srv.release(rid)
    return got


def _inputs(torch, r):
    return (torch.from_numpy(r["xb"]).cuda()[:, :r["n"]], torch.from_numpy(r["m"]).cuda())


def test_serve_alone_equals_mix(orc):
    torch, P = need_gpu()
    reqs = _requests(20, 3)
    dev = [_inputs(torch, r) for r in reqs]
    fps = [P.solve_footprint(_params(P, r), r["n"]) for r in reqs]
    # alone: one slot, every request runs by itself
    alone = []
    with P.Server(max(fps) + (1 << 20), n_streams=1, per_stream=1) as srv:
        for r, (x, m) in zip(reqs, dev):
            rid = srv.submit(_params(P, r), x, m)
            alone.append(_collect(P, torch, srv, [r], [rid], False)[rid])
    # mix: everything submitted at once, 4 streams x 2, arena for about a third
    # of the requests (and at least any two)
    arena = max(2 * max(fps), sum(fps) // 3)
    with P.Server(arena, n_streams=4, per_stream=2) as srv:
        ids = [srv.submit(_params(P, r), x, m) for r, (x, m) in zip(reqs, dev)]
        mix = _collect(P, torch, srv, reqs, ids, False)
        st = srv.stats()
    print("serve stats", st)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["bytes_peak"] <= arena and st["bytes_in_use"] == 0
    assert st["peak_in_flight"] >= 2, "no overlap happened"
    for k, (r, rid) in enumerate(zip(reqs, ids)):
        a, b = alone[k], mix[rid]
        assert a[0]["status"] == 0 and b[0]["status"] == 0
        assert a[0]["soft_interactions"] == b[0]["soft_interactions"]
        assert a[0]["hard_pairs"] == b[0]["hard_pairs"]
        for u, v in zip(a[1:], b[1:]):
            assert (u is None) == (v is None), k
            if u is not None:
                assert torch.equal(u, v), k
    # and the results are the method's: oracle check on the smaller requests
    for k, (r, rid) in enumerate(zip(reqs, ids)):
        if r["n"] > 6000:
            continue
        inf, a_s, a_h, ngb, pot = mix[rid]
        m64 = r["m"].astype(np.float64)
        T = orc.Tree(r["x"], m64, n_crit=16, theta=r["theta"])
        oa, _, oi = T.soft(r["G"], r["eps"], r["R2"] / 2, r["R2"], r["hybrid"])
        e = rel_err(a_s.cpu().numpy().astype(np.float64), oa)
        assert np.percentile(e, 99) <= 1e-5, k
        assert inf["soft_interactions"] == oi, k
        if r["hybrid"]:
            oh, _, ongb = orc.split_direct(r["x"], m64, r["G"], r["eps"], r["R2"] / 2, r["R2"],
                                           soft=False)
            assert np.array_equal(ngb.cpu().numpy(), ongb), k
            eh = rel_err(a_h.cpu().numpy().astype(np.float64), oh)[ongb > 0]
            assert np.percentile(eh, 99) <= 1e-5, k
            assert inf["hard_pairs"] == int(ongb.sum()), k
        else:
            assert a_h is None and ngb is None


def test_serve_waits_for_inputs_written_on_a_side_stream():
    """Inputs written by GPU work on the caller's (side) stream just before
    submission: the solve must read them only after that work."""
    torch, P = need_gpu()
    r = _requests(1, 7, 14.0, 14.0)[0]
    x_host, m_host = _inputs(torch, r)
    with P.Server(P.solve_footprint(_params(P, r), r["n"]) + (1 << 20), 1, 1) as srv:
        rid = srv.submit(_params(P, r), x_host, m_host)
        ref = _collect(P, torch, srv, [r], [rid], False)[rid]
        side = torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            x = torch.zeros_like(x_host)
            m = torch.zeros_like(m_host)
            torch.cuda._sleep(50_000_000)       # keeps the side stream busy
            x.copy_(x_host)
            m.copy_(m_host)
            rid = srv.submit(_params(P, r), x, m)
        got = _collect(P, torch, srv, [r], [rid], False)[rid]
    assert got[0]["status"] == 0
    for u, v in zip(ref[1:], got[1:]):
        assert (u is None) == (v is None)
        if u is not None:
            assert torch.equal(u, v)


def test_serve_admission_and_errors():
    torch, P = need_gpu()
    reqs = _requests(8, 4, 11.0, 13.0)
    dev = [_inputs(torch, r) for r in reqs]
    fps = [P.solve_footprint(_params(P, r), r["n"]) for r in reqs]
    arena = max(fps) + 4096            # one request at a time fits
    with P.Server(arena, n_streams=2, per_stream=2) as srv:
        # never admissible: larger than the arena
        big = _requests(1, 9, 17.0, 17.0)[0]
        xb, mb = _inputs(torch, big)
        with pytest.raises(P.HTreeError) as ei:
            srv.submit(_params(P, big), xb, mb)
        assert ei.value.code == P.HTREE_ENOMEM
        with pytest.raises(P.HTreeError) as ei:
            srv.submit(P.default_params(eps=0.0), dev[0][0], dev[0][1])
        assert ei.value.code == P.HTREE_EINVAL
        ids = [srv.submit(_params(P, r), x, m) for r, (x, m) in zip(reqs, dev)]
        # the last one is normally still queued behind the others: cancel it
        last = ids[-1]
        cancelled = int(srv.info(last)["state"] == P.Server.PENDING)
        if cancelled:
            srv.release(last)
            ids = ids[:-1]
        got = _collect(P, torch, srv, reqs, ids, False)
        st = srv.stats()
    assert st["cancelled"] == cancelled and st["completed"] == len(ids)
    assert st["bytes_peak"] <= arena and st["pending"] == 0 and st["in_flight"] == 0
    for rid in ids:
        inf = got[rid][0]
        assert inf["t_submit"] <= inf["t_admit"] <= inf["t_done"]


def test_serve_trace_small():
    # a short Poisson trace through a generous arena: everything completes,
    # latencies are positive and ordered
    import time
    torch, P = need_gpu()
    rng = np.random.default_rng(5)
    reqs = _requests(60, 6, 10.0, 14.0)
    dev = [_inputs(torch, r) for r in reqs]
    arrivals = np.cumsum(rng.exponential(1 / 2000.0, len(reqs)))
    with P.Server(4 << 30, n_streams=4, per_stream=2) as srv:
        t0 = time.perf_counter()
        ids, lat, k = [], {}, 0
        sub = {}
        while len(lat) < len(reqs):
            now = time.perf_counter() - t0
            assert now < 60.0, "trace did not finish: %s" % srv.stats()
            while k < len(reqs) and arrivals[k] <= now:
                rid = srv.submit(_params(P, reqs[k]), *dev[k])
                sub[rid] = arrivals[k]
                ids.append(rid)
                k += 1
            for rid in srv.poll():
                lat[rid] = time.perf_counter() - t0 - sub[rid]
                srv.release(rid)
        st = srv.stats()
    v = np.array(list(lat.values()))
    print("trace latency p50 %.3f ms p99 %.3f ms, peak in flight %d" %
          (1e3 * np.percentile(v, 50), 1e3 * np.percentile(v, 99), st["peak_in_flight"]))
    assert (v > 0).all() and st["completed"] == len(reqs) and st["held"] == 0
