"""The serving scheduler on the simulated device (no GPU): admission by arena
footprint, FIFO order, work-capped batches, several batches in flight,
cancellation, invalid and never-fitting requests, concurrent submitters and
shutdown with work pending."""
import threading
import time

import pytest

import workloads as W


def _srv(**kw):
    from paper_2606_01547_amd import Server
    cfg = dict(hbm_budget_bytes=64 << 20, max_batch_images=16, max_batch_pairs=5e8, max_inflight_batches=2,
               n_streams=2, simulated_pairs_per_s=1e11)
    cfg.update(kw)
    return Server(None, **cfg)


def _sc(n=64, s=1):
    sc = W.config1_scene()
    sc.grid = W.Grid(nx=n, ny=n, pixel_scale=0.05, supersample=s)
    return sc


def _submit(srv, sc, nsub=100, k=11):
    return srv.submit(sc.grid, sc.lens, sc.source, sc.lens_light, subhalo_handle=nsub, psf_handle=k)


def test_all_requests_complete_in_fifo_order():
    # ~5 ms per job, so every request is queued before the first completes
    srv = _srv(max_inflight_batches=1, max_batch_images=1, simulated_pairs_per_s=1e8)
    sc = _sc()
    tickets = [_submit(srv, sc) for _ in range(20)]
    lat = [srv.wait(t) for t in tickets]
    assert all(b > a for a, b in zip(lat, lat[1:]))   # equal jobs served one at a time, in order
    st = srv.stats()
    assert st["completed"] == 20 and st["batches"] == 20 and st["arena_in_use"] == 0
    srv.close()


def test_batches_pack_waiting_requests_up_to_the_caps():
    srv = _srv(max_batch_images=8, max_inflight_batches=1, simulated_pairs_per_s=1e9)
    sc = _sc()
    first = _submit(srv, sc, nsub=20000)          # occupies the device for ~80 ms
    rest = [_submit(srv, sc, nsub=10) for _ in range(16)]
    srv.wait(first)
    for t in rest:
        srv.wait(t)
    st = srv.stats()
    assert st["completed"] == 17
    assert st["batches"] <= 4                      # 16 small requests in batches of <= 8
    srv.close()


def test_large_request_runs_in_chunks_beside_small_ones():
    # 2.6e10 pairs over a 1e7 cap: 51 429 blocks of 28 pixels in chunks of
    # 2048 blocks (26 chunks) and a convolution launch; the small requests
    # queued behind it are batched while its chunks run (this simulated device
    # runs batches one after another, so they wait for at most the chunks
    # already queued), long before it ends
    srv = _srv(max_batch_pairs=1e7, max_inflight_batches=3)
    t_big = _submit(srv, _sc(1200, 3), nsub=2000)
    small = [_submit(srv, _sc(), nsub=10) for _ in range(5)]
    lat_small = [srv.wait(t) for t in small]
    lat_big = srv.wait(t_big)
    st = srv.stats()
    assert st["completed"] == 6 and st["arena_in_use"] == 0
    assert st["batches"] >= 26 + 1 + 1
    assert max(lat_small) < 0.3 * lat_big
    srv.close()


def test_chunked_requests_beyond_the_stream_limit_wait_in_fifo_order():
    # with 2 streams one chunked request runs at a time: a second waits at the
    # head until the first is done, and the small request behind it waits too
    srv = _srv(max_batch_pairs=1e7, max_inflight_batches=3, n_streams=2)
    big1 = _submit(srv, _sc(600, 3), nsub=2000)     # 12 858 blocks: chunked
    big2 = _submit(srv, _sc(600, 3), nsub=2000)
    small = _submit(srv, _sc(), nsub=10)
    l1, l2, ls = srv.wait(big1), srv.wait(big2), srv.wait(small)
    assert 0.5 * l1 < ls < l2          # it waited for the first large request, not the second
    assert srv.stats()["completed"] == 3
    srv.close()


def test_several_chunked_requests_run_together():
    # with 4 streams up to 3 chunked requests are in progress at once, so the
    # small request behind two of them is not held until they finish
    srv = _srv(max_batch_pairs=1e7, max_inflight_batches=4, n_streams=4)
    big = [_submit(srv, _sc(600, 3), nsub=2000) for _ in range(2)]
    small = _submit(srv, _sc(), nsub=10)
    ls = srv.wait(small)
    lb = [srv.wait(t) for t in big]
    assert ls < 0.5 * min(lb)
    assert srv.stats()["completed"] == 3 and srv.stats()["arena_in_use"] == 0
    srv.close()


def test_request_over_the_cap_with_few_blocks_runs_alone():
    # 120^2, s = 3: 2058 blocks, too few to chunk; over the cap it forms a
    # batch of its own instead of joining the small ones
    srv = _srv(max_batch_pairs=1e7, max_inflight_batches=1, max_batch_images=16)
    ts = [_submit(srv, _sc(120, 3), nsub=2000) for _ in range(3)]
    for t in ts:
        srv.wait(t)
    assert srv.stats()["batches"] == 3
    srv.close()


def test_admission_waits_for_arena_space():
    sc = _sc(400, 3)
    from paper_2606_01547_amd import Server
    one = 4 * 400 * 400 + (400 * 400 // 7) * 8 + 13 * 50 * 16 + 4096
    srv = Server(None, hbm_budget_bytes=int(1.5 * one), max_batch_images=8, max_batch_pairs=1e15,
                 max_inflight_batches=4, n_streams=4, simulated_pairs_per_s=1e13)
    ts = [_submit(srv, sc, nsub=100, k=41) for _ in range(5)]
    for t in ts:
        srv.wait(t)
    st = srv.stats()
    assert st["batches"] == 5                       # one at a time fits the arena
    assert st["arena_peak"] <= st["arena_bytes"]
    srv.close()


def test_never_fitting_and_invalid_requests_are_rejected():
    from paper_2606_01547_amd import JtError
    from paper_2606_01547_amd._native import JT_EINVAL, JT_ENOMEM
    srv = _srv(hbm_budget_bytes=1 << 16)
    with pytest.raises(JtError) as e:
        _submit(srv, _sc(400, 3), k=41)
    assert e.value.status == JT_ENOMEM
    bad = _sc()
    bad.lens.sie = W.SIE(1.0, 1.5, 0.0, 0.0, 0.0)
    with pytest.raises(JtError) as e:
        _submit(srv, bad)
    assert e.value.status == JT_EINVAL
    with pytest.raises(JtError) as e:
        _submit(srv, _sc(), k=4)
    assert e.value.status == JT_EINVAL
    with pytest.raises(JtError):
        srv.wait(12345)
    srv.close()


def test_cancel_queued_ticket():
    from paper_2606_01547_amd import JtError
    from paper_2606_01547_amd._native import JT_ECANCELLED, TICKET_QUEUED
    srv = _srv(max_inflight_batches=1, max_batch_images=1, simulated_pairs_per_s=1e9)
    sc = _sc(200, 3)
    a = _submit(srv, sc, nsub=5000)
    b = _submit(srv, sc, nsub=5000)
    assert srv.poll(b) == TICKET_QUEUED
    srv.cancel(b)
    with pytest.raises(JtError) as e:
        srv.wait(b)
    assert e.value.status == JT_ECANCELLED
    srv.wait(a)
    assert srv.stats()["cancelled"] == 1
    srv.close()


def test_concurrent_submitters():
    srv = _srv(max_batch_images=32, max_inflight_batches=3)
    sc = _sc()
    out = []
    lock = threading.Lock()

    def worker():
        mine = [_submit(srv, sc, nsub=50) for _ in range(25)]
        for t in mine:
            srv.wait(t)
        with lock:
            out.extend(mine)

    th = [threading.Thread(target=worker) for _ in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert len(set(out)) == 100 and srv.stats()["completed"] == 100
    srv.close()


def test_destroy_with_pending_work_cancels_the_queue():
    srv = _srv(max_inflight_batches=1, max_batch_images=1, simulated_pairs_per_s=1e9)
    sc = _sc(200, 3)
    for _ in range(10):
        _submit(srv, sc, nsub=2000)
    t0 = time.time()
    srv.close()
    assert time.time() - t0 < 5.0


def test_injected_device_failure_fails_in_flight_and_queued_and_refuses_submits():
    """Batch 3 fails on the (simulated) device: tickets 1-2 completed before
    it are done; 3, the batch in flight beside it and everything queued fail
    (JT_EDEVICE); later submissions are refused; the arena drains."""
    from paper_2606_01547_amd import JtError
    from paper_2606_01547_amd._native import JT_EDEVICE
    srv = _srv(max_inflight_batches=2, max_batch_images=1, n_streams=2, simulated_pairs_per_s=1e9)
    srv.simulate_failure(3)
    sc = _sc(100, 1)
    tickets = [_submit(srv, sc, nsub=2000) for _ in range(10)]      # ~20 ms each, one per batch
    ok, failed = [], []
    for t in tickets:
        try:
            srv.wait(t, timeout=30.0)
            ok.append(t)
        except JtError as e:
            assert e.status == JT_EDEVICE, e
            failed.append(t)
    assert ok == tickets[:2] and failed == tickets[2:]
    with pytest.raises(JtError) as e:
        _submit(srv, sc)
    assert e.value.status == JT_EDEVICE and "device failure" in str(e.value)
    st = srv.stats()
    assert st["completed"] == 2 and st["failed"] == 8 and st["batches"] <= 4
    assert st["arena_in_use"] == 0
    srv.close()


def test_injected_failure_inside_a_chunked_request():
    """The second chunk of a large request fails: the request fails once its
    launched chunks are done, without launching more chunks or its
    convolution; small requests that ran beside it on another stream before
    the failure completed, the rest fail, and later submissions are refused."""
    from paper_2606_01547_amd import JtError
    from paper_2606_01547_amd._native import JT_EDEVICE
    # chunks of ~0.5 s, so that the three small requests are submitted well
    # before the failing second chunk ends, even on a loaded host
    srv = _srv(max_batch_pairs=1e7, max_inflight_batches=3, n_streams=2, simulated_pairs_per_s=2e9)
    srv.simulate_failure(2)
    big = _submit(srv, _sc(1200, 3), nsub=2000)                        # 26 chunks of ~0.5 s + a convolution
    small = []
    for sc in [_sc() for _ in range(3)]:
        try:
            small.append(_submit(srv, sc, nsub=10))
        except JtError as e:      # only if this thread stalled past the failure (a loaded host)
            assert e.status == JT_EDEVICE
    with pytest.raises(JtError) as e:
        srv.wait(big, timeout=30.0)
    assert e.value.status == JT_EDEVICE
    outcome = []
    for t in small:
        try:
            srv.wait(t, timeout=30.0)
            outcome.append("done")
        except JtError as e:
            assert e.status == JT_EDEVICE
            outcome.append("failed")
    with pytest.raises(JtError) as e:
        _submit(srv, _sc(), nsub=10)
    assert e.value.status == JT_EDEVICE
    st = srv.stats()
    assert st["failed"] == 1 + outcome.count("failed") and st["completed"] == outcome.count("done")
    assert st["batches"] < 8                    # of the 27 launches the request needs, at most its first 3 ran
    assert st["arena_in_use"] == 0
    srv.close()


def test_destroy_cancels_a_chunked_request_in_progress():
    """Closing the server while a chunked request runs launches no further
    chunk; a thread waiting on its ticket is released with JT_ECANCELLED
    before the server is freed."""
    from paper_2606_01547_amd import JtError
    from paper_2606_01547_amd._native import JT_ECANCELLED, TICKET_RUNNING
    srv = _srv(max_batch_pairs=1e7, max_inflight_batches=3, n_streams=2, simulated_pairs_per_s=1e9)
    big = _submit(srv, _sc(1200, 3), nsub=2000)                        # ~26 s of simulated work
    t0 = time.time()
    while srv.poll(big) != TICKET_RUNNING:
        assert time.time() - t0 < 5.0
        time.sleep(1e-3)
    seen = []

    def waiter():
        try:
            srv.wait(big)
            seen.append("done")
        except JtError as e:
            seen.append(e.status)

    th = threading.Thread(target=waiter)
    th.start()
    time.sleep(0.05)
    t0 = time.time()
    srv.close()
    th.join(timeout=10.0)
    assert not th.is_alive()
    assert seen == [JT_ECANCELLED]
    assert time.time() - t0 < 5.0               # two queued chunks of ~1 s at most, not the whole image
