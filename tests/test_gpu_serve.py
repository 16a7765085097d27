"""GPU: the serving loop (continuous batching). Requests of both kinds and uneven sizes are
submitted while others are in flight; every result matches the float64 oracle (with and without
the block preconditioner), is the same alone and in the mix, and admission respects the
device-memory budget."""
import threading
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import nystrom as ny  # noqa: E402
from paper_1507_05925_amd import bie2d  # noqa: E402
from paper_1507_05925_amd import workloads as wl  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs the GPU")]


def sessions():
    rng = np.random.default_rng(31)
    out = []
    for i in range(6):
        N = int(rng.integers(2, 12))
        nodes = 32 * rng.integers(2, 9, size=N)
        c = wl.mixed_grid(rng, N, nodes)
        kind = 0 if i % 5 < 3 else 1
        nq = int(rng.integers(1, 4))
        width = N if kind == 0 else 3 * N
        qs = [rng.standard_normal((int(rng.integers(1, 3)), width)) for _ in range(nq)]
        out.append((kind, c, qs))
    return out


def oracle_answers(sess):
    ans = []
    for kind, c, qs in sess:
        geo = ny.geometry_of(c)
        f = ny.elastance_solve if kind == 0 else ny.mobility_solve
        key = "phi" if kind == 0 else "VW"
        ans.append([f(geo, q)[key] for q in qs])
    return ans


@pytest.mark.parametrize("precond", [bie2d.BIE_PRECOND_NONE, bie2d.BIE_PRECOND_BLOCK])
@pytest.mark.parametrize("precision,tol", [(bie2d.BIE_FP64, 1e-10), (bie2d.BIE_MIXED, 1e-9)])
def test_serve_mix_matches_oracle_and_alone(precision, tol, precond):
    sess = sessions()
    ref = oracle_answers(sess)
    opts = bie2d.default_opts(precision=precision, tol=1e-12, restart=30, precond=precond)
    geoms = [bie2d.Geometry.from_curves(c) for _, c, _ in sess]
    # in the mix: submit everything from two threads with small random gaps
    srv = bie2d.Server(opts)
    tickets = {}
    lock = threading.Lock()

    def client(idx):
        rng = np.random.default_rng(100 + idx)
        for si in range(idx, len(sess), 2):
            for qi, q in enumerate(sess[si][2]):
                t = srv.submit(geoms[si], sess[si][0], q)
                with lock:
                    tickets[(si, qi)] = t
                time.sleep(float(rng.uniform(0, 0.002)))

    th = [threading.Thread(target=client, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    mix = {}
    for key, t in tickets.items():
        out, info = srv.wait(t, timeout=120)
        assert info["status"] == 0 and info["rel_residual"] <= 1e-12, info
        mix[key] = out
    st = srv.stats()
    srv.close()
    assert st["requests"] == len(tickets)
    for (si, qi), out in mix.items():
        r = ref[si][qi]
        assert float(np.abs(out - r).max() / np.abs(r).max()) < tol, (si, qi)
    # alone: a fresh server, one request at a time
    srv = bie2d.Server(opts)
    for (si, qi), out in mix.items():
        t = srv.submit(geoms[si], sess[si][0], sess[si][2][qi])
        alone, _ = srv.wait(t, timeout=120)
        assert np.array_equal(alone, out), (si, qi)
    srv.close()


def test_serve_budget_limits_concurrency():
    """Admission by device-memory footprint: with a budget of one byte every request runs
    alone (a request is always admitted when nothing else is in flight) and the bytes in flight
    never exceed the largest single footprint; without a budget the same submissions overlap."""
    sess = sessions()[:4]
    geoms = [bie2d.Geometry.from_curves(c) for _, c, _ in sess]
    opts = bie2d.default_opts(precision=bie2d.BIE_MIXED, tol=1e-11, restart=20)
    peaks = {}
    for budget in (1, 0):
        srv = bie2d.Server(opts, hbm_budget_bytes=budget)
        tks = []
        for (kind, c, qs), g in zip(sess, geoms):
            for q in qs:
                tks.append((srv.submit(g, kind, q), kind, c, q))
        infl, foot = [], []
        for t, kind, c, q in tks:
            out, info = srv.wait(t, timeout=120)
            assert info["status"] == 0
            infl.append(info["inflight"])
            foot.append(info["footprint_bytes"])
            geo = ny.geometry_of(c)
            ref = ny.elastance_solve(geo, q)["phi"] if kind == 0 else ny.mobility_solve(geo, q)["VW"]
            assert float(np.abs(out - ref).max() / np.abs(ref).max()) < 1e-9
        st = srv.stats()
        srv.close()
        assert st["requests"] == len(tks)
        peaks[budget] = (max(infl), st["peak_bytes"], max(foot))
    assert peaks[1][0] == 1 and peaks[1][1] <= peaks[1][2], peaks
    assert peaks[0][0] >= 2, peaks


def test_serve_failed_cycle_fails_only_its_requests():
    """An internal error in a cycle (injected from the host) fails the requests in flight in
    that cycle; the worker stays up and a later request completes and matches the oracle."""
    sess = sessions()
    kind, c, qs = sess[0]
    g = bie2d.Geometry.from_curves(c)
    geo = ny.geometry_of(c)
    ref = ny.elastance_solve(geo, qs[0])["phi"] if kind == 0 else ny.mobility_solve(geo, qs[0])["VW"]
    srv = bie2d.Server(bie2d.default_opts(tol=1e-12, restart=30))
    out, info = srv.wait(srv.submit(g, kind, qs[0]), timeout=120)
    assert info["status"] == 0
    srv.inject_failure(1)
    out, info = srv.wait(srv.submit(g, kind, qs[0]), timeout=120, raise_on_error=False)
    assert info["status"] == bie2d.BIE_EDEVICE, info
    out, info = srv.wait(srv.submit(g, kind, qs[0]), timeout=120)
    assert info["status"] == 0
    assert float(np.abs(out - ref).max() / np.abs(ref).max()) < 1e-10
    assert srv.stats()["requests"] == 2
    srv.close()


def test_serve_precond_refusal_fails_only_that_request():
    """With the block preconditioner, a request on a geometry whose bodies it cannot coarsen (a
    body of 257 nodes: no divisor in [16, 64]) fails alone with BIE_EINVAL while it is being
    admitted; a request submitted beside it completes and matches the oracle."""
    rng = np.random.default_rng(47)
    bad = bie2d.Geometry.from_curves(wl.mixed_grid(rng, 3, np.array([64, 257, 96])))
    kind, c, qs = sessions()[0]
    good = bie2d.Geometry.from_curves(c)
    geo = ny.geometry_of(c)
    ref = ny.elastance_solve(geo, qs[0])["phi"] if kind == 0 else ny.mobility_solve(geo, qs[0])["VW"]
    srv = bie2d.Server(bie2d.default_opts(tol=1e-12, restart=30, precond=bie2d.BIE_PRECOND_BLOCK))
    tb = srv.submit(bad, 0, rng.standard_normal((1, 3)))
    tg = srv.submit(good, kind, qs[0])
    _, info = srv.wait(tb, timeout=120, raise_on_error=False)
    assert info["status"] == bie2d.BIE_EINVAL, info
    out, info = srv.wait(tg, timeout=120)
    assert info["status"] == 0
    assert float(np.abs(out - ref).max() / np.abs(ref).max()) < 1e-10
    srv.close()
