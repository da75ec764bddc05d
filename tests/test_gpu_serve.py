"""GPU serving loop: requests from many client threads are batched with others
of different size, and every result equals the event run alone through
trk_event (the analogue of the paper's check that track candidates are the same
whether inference runs locally or through the server, Section 4.2)."""
import threading

import numpy as np
import pytest

from gen import TINY, MU200, make_weights, generate_event

pytestmark = pytest.mark.gpu


def _serve_many(srv, xs, n_threads):
    results = [None] * len(xs)

    def client(k0):
        for k in range(k0, len(xs), n_threads):
            t = srv.submit(xs[k])
            results[k] = srv.wait(t, xs[k].shape[0])

    th = [threading.Thread(target=client, args=(c,)) for c in range(n_threads)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    return results


def test_tiny_mix_equals_alone():
    from paper_2501_05520_amd.trk import Server, Pipeline
    nets = make_weights(TINY, 0)
    xs = [generate_event(s, 1 + s % 3).x for s in range(1, 25)]      # 550, 1100, 1650 hits
    srv = Server(TINY, nets, "fp32", n_slots=2, max_batch_events=4, max_batch_hits=6000)
    res = _serve_many(srv, xs, 8)
    st = srv.stats()
    srv.close()
    pipe = Pipeline(TINY, nets, "fp32", max_hits=6000)
    for x, (rc, labels, info, lat) in zip(xs, res):
        assert rc == 0
        alone, ainfo = pipe.event(x)
        assert np.array_equal(labels, alone.cpu().numpy())
        assert info["n_cand_edges"] == ainfo["n_cand_edges"] and lat > 0
    pipe.close()
    assert st["completed"] == len(xs) and st["batches"] < len(xs)


@pytest.mark.parametrize("precision", ["bf16", "bf16x3", "fp8"])
def test_mu_mix_equals_alone(precision):
    from paper_2501_05520_amd.trk import Server, Pipeline
    nets = make_weights(MU200, 0)
    xs = [generate_event(400 + k, mu).x for k, mu in enumerate((50, 100, 140, 50, 100, 140))]
    srv = Server(MU200, nets, precision, n_slots=2, max_batch_events=4, max_batch_hits=160000)
    res = _serve_many(srv, xs, 6)
    st = srv.stats()
    srv.close()
    pipe = Pipeline(MU200, nets, precision, max_hits=80000)
    for x, (rc, labels, info, lat) in zip(xs, res):
        assert rc == 0
        alone, _ = pipe.event(x)
        assert np.array_equal(labels, alone.cpu().numpy())
    pipe.close()
    assert st["completed"] == len(xs)


def test_admission_refuses_oversized_and_reports():
    from paper_2501_05520_amd import trk
    nets = make_weights(TINY, 0)
    srv = trk.Server(TINY, nets, "fp32", n_slots=1, max_batch_events=2, max_batch_hits=1000,
                     mem_budget_bytes=1 << 40)
    x = generate_event(1, 2).x                      # 1100 hits > max_batch_hits
    with pytest.raises(trk.TrkError) as e:
        srv.submit(x)
    assert e.value.status == -3
    t = srv.submit(x[:500])
    rc, labels, info, lat = srv.wait(t, 500)
    assert rc == 0 and info["n_hits"] == 500
    srv.close()


def test_socket_front_end_equals_alone():
    """Requests through the TCP front end (several connections at once) return the
    labels trk_event gives each event alone."""
    from paper_2501_05520_amd import trk
    from paper_2501_05520_amd.trk import Server, Pipeline, ServiceClient
    nets = make_weights(TINY, 0)
    xs = [generate_event(s, 1 + s % 2).x for s in range(30, 46)]
    srv = Server(TINY, nets, "fp32", n_slots=2, max_batch_events=4, max_batch_hits=6000)
    svc, port = trk.trk_service_start(srv.h, "127.0.0.1", 0)
    results = [None] * len(xs)

    def client(c):
        cl = ServiceClient("127.0.0.1", port)
        for k in range(c, len(xs), 4):
            results[k] = cl.request(xs[k])
        cl.close()

    th = [threading.Thread(target=client, args=(c,)) for c in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    bad = ServiceClient("127.0.0.1", port).request(np.zeros((7000, 3), np.float32))   # beyond max_batch_hits
    trk.trk_service_stop(svc)
    srv.close()
    assert bad[0] == -1
    pipe = Pipeline(TINY, nets, "fp32", max_hits=6000)
    for x, (status, labels, info, lat) in zip(xs, results):
        alone, ainfo = pipe.event(x)
        assert status == 0 and np.array_equal(labels, alone.cpu().numpy())
        assert info["n_cand_edges"] == ainfo["n_cand_edges"] and lat > 0
    pipe.close()
