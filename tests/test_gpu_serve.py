"""Continuous-batching server: results match the FP64 oracle run with the
same subset sequence, each result is bitwise the same alone and in the mix,
admission respects slots and the memory budget, cancellation works."""

import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2106_03172_amd as pkg  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


SPECS = [  # (nx, views, bins, subsets, counts, seed)
    (48, 40, 67, 8, 5e4, 31),
    (64, 60, 87, 6, 1e5, 32),
    (32, 30, 45, 5, 3e4, 33),
    (56, 50, 77, 10, 8e4, 34),
]
EPOCHS, ALPHA, BETA = 3, 0.7, 1e-3


def _req(spec):
    nx, V, B, Ns, counts, seed = spec
    return datagen.make_problem(nx, nx, 2.0, V, B, 2.0, Ns, counts, seed=seed)


def _serve(problems, max_slots=8, budget=1 << 31, seeds=None):
    S = pkg.Server(budget, max_slots=max_slots, n_streams=3)
    tickets = []
    for i, P in enumerate(problems):
        prm = pkg.params("svrem", alpha=ALPHA, eta=1, beta=BETA)
        tickets.append(S.submit(P.geom, P.n_subsets, P.g, P.w, prm, EPOCHS,
                                order_seed=(seeds[i] if seeds else 1000 + i)))
    S.step(0)
    res = [S.poll(t) for t in tickets]
    S.close()
    return res


def test_server_matches_oracle_and_direct_recon():
    P = _req(SPECS[1])
    r = _serve([P], seeds=[77])[0]
    assert r["status"] == 0
    orders = pkg.splitmix64_orders(77, P.n_subsets, EPOCHS)
    # direct recon through the C ABI with the same subset sequence: bitwise equal
    A = pkg.SystemMatrix(P.geom, P.n_subsets)
    R = pkg.Recon(A, P.g, P.w, np.ones((1, P.geom.n_pixels)), pkg.params("svrem", alpha=ALPHA, eta=1, beta=BETA))
    R.osem_epoch(list(range(P.n_subsets)))
    for o in orders:
        R.svrem_epoch(o)
    np.testing.assert_array_equal(r["f"], R.image().cpu().numpy()[0])
    # FP64 oracle
    Ao = oracle.system_matrix(P.geom)
    m = oracle.Model(Ao, P.g, P.w, P.geom, P.n_subsets, beta=BETA)
    f = oracle.osem_epoch(m, np.ones((1, P.geom.n_pixels)), range(P.n_subsets))
    alg = oracle.SVREM(m, f, ALPHA, 1)
    for o in orders:
        alg.run(o)
    assert rel(r["f"], alg.f) <= 1e-5
    assert abs(r["phi"] - m.objective(r["f"][None, :].astype(np.float64))) <= 1e-6 * abs(r["phi"])


@pytest.mark.parametrize("wtype,bar", [(pkg.SVR_W_F32, 1e-5), (pkg.SVR_W_F16, 1e-3), (pkg.SVR_W_BF16, 2.5e-3)])
def test_thirty_epochs_served_against_oracle(wtype, bar):
    """A serving request's 30 SVREM epochs against the FP64 oracle run with
    the same subset sequence: FP32 weights within the parity bar, FP16
    weights within 1e-3 (the error bar at which a half-precision batched
    serving form is compared with the plain FP32 per-request path).  BF16
    weights (8 significant bits) end at 1.8e-3 here: their rounding shifts
    the fixed point the iteration approaches; bounded at 2.5e-3."""
    P = _req(SPECS[1])
    S = pkg.Server(1 << 31, max_slots=2, n_streams=2)
    prm = pkg.params("svrem", alpha=ALPHA, eta=1, beta=BETA)
    t = S.submit(P.geom, P.n_subsets, P.g, P.w, prm, 30, order_seed=91, wtype=wtype)
    S.step(0)
    r = S.poll(t)
    S.close()
    assert r["status"] == 0
    Ao = oracle.system_matrix(P.geom)
    m = oracle.Model(Ao, P.g, P.w, P.geom, P.n_subsets, beta=BETA)
    alg = oracle.SVREM(m, oracle.osem_epoch(m, np.ones((1, P.geom.n_pixels)), range(P.n_subsets)), ALPHA, 1)
    for o in pkg.splitmix64_orders(91, P.n_subsets, 30):
        alg.run(o)
    err = rel(r["f"], alg.f)
    print("rel L2 vs oracle after 30 epochs", wtype, err, flush=True)
    assert err <= bar


def test_batched_kernels_equal_per_request_streams():
    """batch = 1 runs the subset iterations of all resident requests of one
    storage type as one forward and one update launch; every request's result
    must be bitwise the one of the per-request path (batch = 0), across a mix
    of FP32, BF16 and FP16 weights and of 16- and 32-bit indices (two type
    groups run their own launches), with more requests than one launch holds."""
    probs = [_req(s) for s in SPECS] * 3
    wts = [pkg.SVR_W_F32, pkg.SVR_W_BF16, pkg.SVR_W_F32 | pkg.binding.SVR_W_INDEX32, pkg.SVR_W_F16] * 3
    prm = pkg.params("svrem", alpha=ALPHA, eta=1, beta=BETA)
    out = []
    for batch in (True, False):
        S = pkg.Server(1 << 32, max_slots=12, n_streams=3, batch=batch)
        tk = [S.submit(P.geom, P.n_subsets, P.g, P.w, prm, EPOCHS, 500 + i, wtype=wts[i])
              for i, P in enumerate(probs)]
        S.step(0)
        out.append([S.poll(t) for t in tk])
        S.close()
    for a, b in zip(*out):
        assert a["status"] == 0 and b["status"] == 0
        np.testing.assert_array_equal(a["f"], b["f"])
        assert a["phi"] == b["phi"]
    # a batching server runs the per-phase kernels only
    S = pkg.Server(1 << 31, max_slots=2, n_streams=1, batch=True)
    with pytest.raises(pkg.SvrError):
        S.submit(probs[0].geom, probs[0].n_subsets, probs[0].g, probs[0].w,
                 pkg.params("svrem", flags=pkg.binding.FLAG_PERSISTENT_EPOCH), 2, 1)
    S.close()


def test_alone_equals_in_the_mix():
    probs = [_req(s) for s in SPECS]
    mixed = _serve(probs, max_slots=3, seeds=[11, 12, 13, 14])
    for i, P in enumerate(probs):
        alone = _serve([P], seeds=[11 + i])[0]
        np.testing.assert_array_equal(alone["f"], mixed[i]["f"])
        assert alone["phi"] == mixed[i]["phi"]


def test_admission_by_slots_and_budget():
    probs = [_req(s) for s in SPECS[:3]]
    res = _serve(probs, max_slots=1)
    assert all(r["status"] == 0 for r in res)
    # one slot: each later request waited for the earlier ones
    assert res[1]["queue_ms"] >= res[0]["run_ms"] * 0.5
    assert res[2]["queue_ms"] >= res[1]["queue_ms"]
    # a request that can never fit the budget is rejected at submit
    S = pkg.Server(1 << 20, max_slots=2, n_streams=1)
    with pytest.raises(pkg.SvrError):
        S.submit(probs[0].geom, probs[0].n_subsets, probs[0].g, probs[0].w, pkg.params("svrem"), 2, 1)
    S.close()


def test_cancel_and_unknown_ticket():
    probs = [_req(s) for s in SPECS[:2]]
    S = pkg.Server(1 << 31, max_slots=1, n_streams=1)
    prm = pkg.params("svrem", alpha=ALPHA, eta=1, beta=BETA)
    t0 = S.submit(probs[0].geom, probs[0].n_subsets, probs[0].g, probs[0].w, prm, EPOCHS, 1)
    t1 = S.submit(probs[1].geom, probs[1].n_subsets, probs[1].g, probs[1].w, prm, EPOCHS, 2)
    S.cancel(t1)
    S.step(0)
    assert S.poll(t0)["status"] == 0
    assert S.poll(t1)["status"] == pkg.binding.SVR_ECANCELLED
    with pytest.raises(pkg.SvrError):
        S.poll(12345)
    S.close()


@pytest.mark.parametrize("batch", [True, False])
def test_server_stats_track_queue_slots_memory_and_totals(batch):
    """svr_serve_stats: after submits everything is queued; a tick admits up
    to max_slots requests, whose held bytes stay within the budget; a cancelled
    request counts as completed; when all are done nothing is held, every
    admitted request is completed, the epochs are the requests' epochs and the
    results wait unpolled until polled."""
    probs = [_req(s) for s in SPECS]
    budget = 1 << 31
    S = pkg.Server(budget, max_slots=2, n_streams=2, batch=batch)
    prm = pkg.params("svrem", alpha=ALPHA, eta=1, beta=BETA)
    tickets = [S.submit(P.geom, P.n_subsets, P.g, P.w, prm, EPOCHS, 50 + i) for i, P in enumerate(probs)]
    st = S.stats()
    assert (st["queued"], st["resident"], st["max_slots"], st["done_unpolled"]) == (4, 0, 2, 0)
    assert (st["used_bytes"], st["mem_budget_bytes"], st["ticks"], st["admitted"], st["completed"]) == \
        (0, budget, 0, 0, 0)
    S.cancel(tickets[3])
    st = S.stats()
    assert (st["queued"], st["completed"], st["done_unpolled"]) == (3, 1, 1)
    S.step(1)  # no request resident yet: the tick admits two
    st = S.stats()
    assert (st["queued"], st["resident"], st["admitted"], st["ticks"]) == (1, 2, 2, 1)
    assert 0 < st["used_bytes"] <= budget
    S.step(0)
    st = S.stats()
    assert (st["queued"], st["resident"], st["used_bytes"]) == (0, 0, 0)
    assert (st["admitted"], st["completed"], st["done_unpolled"]) == (3, 4, 4)
    assert st["epochs"] == 3 * EPOCHS
    for t in tickets[:3]:
        assert S.poll(t)["status"] == 0
    assert S.poll(tickets[3])["status"] == pkg.binding.SVR_ECANCELLED
    assert S.stats()["done_unpolled"] == 0
    S.close()


@pytest.mark.parametrize("batch", [True, False])
def test_kept_blocks_are_reused_and_results_do_not_change(batch):
    """The device blocks of finished requests stay in the server's cache and
    serve later admissions: a second round of the same requests on the same
    server (in a different order, so blocks land in other roles) reuses them,
    holds no more than the budget, and every image and objective is bitwise
    the first round's (nothing depends on what a reused block held)."""
    probs = [_req(s) for s in SPECS]
    budget = 1 << 31
    S = pkg.Server(budget, max_slots=4, n_streams=2, batch=batch)
    prm = pkg.params("svrem", alpha=ALPHA, eta=1, beta=BETA)

    def round_(order):
        t = {i: S.submit(probs[i].geom, probs[i].n_subsets, probs[i].g, probs[i].w, prm, EPOCHS, 300 + i)
             for i in order}
        S.step(0)
        return {i: S.poll(t[i]) for i in order}

    first = round_([0, 1, 2, 3])
    st = S.stats()
    assert st["used_bytes"] == 0 and st["cached_bytes"] > 0 and st["block_reuses"] == 0
    assert st["cached_bytes"] <= budget
    second = round_([3, 1, 0, 2])
    st = S.stats()
    assert st["block_reuses"] > 0 and st["used_bytes"] == 0 and st["cached_bytes"] <= budget
    for i in range(4):
        assert first[i]["status"] == 0 and second[i]["status"] == 0
        np.testing.assert_array_equal(first[i]["f"], second[i]["f"])
        assert first[i]["phi"] == second[i]["phi"]
    S.close()


def test_cache_yields_to_the_budget():
    """Kept blocks count against the budget: with room for about one request,
    each admission first frees kept blocks, so used_bytes + cached_bytes stays
    within the budget after every tick, and every request finishes."""
    probs = [_req(SPECS[1]), _req(SPECS[3])]
    prm = pkg.params("svrem", alpha=ALPHA, eta=1, beta=BETA)
    held = []
    for k, P in enumerate(probs):  # what each request leaves in the cache when run alone
        S = pkg.Server(1 << 31, max_slots=1, n_streams=1)
        t = S.submit(P.geom, P.n_subsets, P.g, P.w, prm, EPOCHS, 1 + k)
        S.step(0)
        assert S.poll(t)["status"] == 0
        held.append(S.stats()["cached_bytes"])
        S.close()
    budget = 3 * max(held)  # the admission estimate runs at about twice what a small request holds
    S = pkg.Server(budget, max_slots=1, n_streams=1)
    ts = [S.submit(P.geom, P.n_subsets, P.g, P.w, prm, EPOCHS, 5 + i) for i, P in enumerate(probs * 2)]
    peak = 0
    while S.stats()["completed"] < len(ts):
        S.step(1)
        st = S.stats()
        assert st["used_bytes"] + st["cached_bytes"] <= budget
        peak = max(peak, st["cached_bytes"])
    assert peak > 0
    assert all(S.poll(t)["status"] == 0 for t in ts)
    S.close()


def test_done_lists_finished_unpolled_tickets():
    """svr_serve_done: nothing before a tick; afterwards exactly the finished,
    unpolled tickets in ascending order (a cancelled one included), capped by
    cap; a polled ticket leaves the list.  A cancelled request's image polls
    as zeros."""
    probs = [_req(s) for s in SPECS[:3]]
    S = pkg.Server(1 << 31, max_slots=1, n_streams=1)
    prm = pkg.params("svrem", alpha=ALPHA, eta=1, beta=BETA)
    tk = [S.submit(P.geom, P.n_subsets, P.g, P.w, prm, 1, 70 + i) for i, P in enumerate(probs)]
    assert S.done() == []
    S.cancel(tk[2])
    assert S.done() == [tk[2]]
    r = S.poll(tk[2])
    assert r["status"] == pkg.binding.SVR_ECANCELLED and not np.any(r["f"])
    S.step(0)
    assert S.done() == tk[:2] and S.done(cap=1) == tk[:1] and S.done(cap=0) == []
    first = S.poll(tk[0])
    assert first["status"] == 0 and np.all(np.isfinite(first["f"])) and first["f"].max() > 0
    assert S.done() == [tk[1]]
    assert S.poll(tk[1])["status"] == 0 and S.done() == []
    S.close()


@pytest.mark.parametrize("batch", [True, False])
def test_many_concurrent_admissions_match_requests_alone(batch):
    """Twelve requests admitted in one tick (one host thread each, four
    threads to a stream on three streams) end bitwise as each does served
    alone."""
    specs = [(nx, V, B, Ns, c, 400 + k) for k, (nx, V, B, Ns, c, _) in enumerate(SPECS * 3)]
    probs = [_req(s) for s in specs]
    prm = pkg.params("svrem", alpha=ALPHA, eta=1, beta=BETA)
    S = pkg.Server(1 << 31, max_slots=12, n_streams=3, batch=batch)
    tk = [S.submit(P.geom, P.n_subsets, P.g, P.w, prm, EPOCHS, 600 + i) for i, P in enumerate(probs)]
    S.step(1)
    assert S.stats()["admitted"] == 12
    S.step(0)
    mixed = [S.poll(t) for t in tk]
    S.close()
    for i, P in enumerate(probs):
        alone = _serve([P], seeds=[600 + i])[0]
        assert mixed[i]["status"] == 0 and alone["status"] == 0
        np.testing.assert_array_equal(mixed[i]["f"], alone["f"])
        assert mixed[i]["phi"] == alone["phi"]


@pytest.mark.parametrize("batch", [True, False])
def test_requests_of_one_geometry_share_a_matrix(batch):
    """Requests with the same geometry, subset count and weight type (one
    scanner, different data) use one matrix: built once, kept idle after its
    last user finishes and used again by a later request, while each image and
    objective stays bitwise what a server without sharing gives."""
    nx, V, B, Ns = 48, 40, 67, 8
    probs = [datagen.make_problem(nx, nx, 2.0, V, B, 2.0, Ns, c, seed=700 + k)
             for k, c in enumerate([3e4, 5e4, 8e4, 2e4, 6e4])]
    prm = pkg.params("svrem", alpha=ALPHA, eta=1, beta=BETA)

    def serve(share):
        S = pkg.Server(1 << 31, max_slots=3, n_streams=2, batch=batch, share_matrices=share)
        tk = [S.submit(P.geom, P.n_subsets, P.g, P.w, prm, EPOCHS, 800 + i) for i, P in enumerate(probs[:4])]
        S.step(0)
        out = [S.poll(t) for t in tk]
        st = S.stats()
        late = S.submit(probs[4].geom, probs[4].n_subsets, probs[4].g, probs[4].w, prm, EPOCHS, 804)
        S.step(0)
        out.append(S.poll(late))
        st2 = S.stats()
        S.close()
        return out, st, st2

    shared, st, st2 = serve(True)
    own, st_own, st_own2 = serve(False)
    assert st["matrix_reuses"] == 3 and st2["matrix_reuses"] == 4  # one build for all five
    assert st["used_bytes"] == 0 and st["cached_bytes"] > 0
    assert st_own["matrix_reuses"] == 0 and st_own2["matrix_reuses"] == 0
    for a, b in zip(shared, own):
        assert a["status"] == 0 and b["status"] == 0
        np.testing.assert_array_equal(a["f"], b["f"])
        assert a["phi"] == b["phi"]


@pytest.mark.parametrize("eta", [1, 2])
def test_batched_anchors_equal_direct_recons(eta):
    """Three requests of one storage type (so their anchors run as shared
    batched launches) with anchors every eta epochs end bitwise as the same
    requests run through the direct epoch calls with the server's subset
    sequences (the anchor of the first iteration of every eta-th epoch)."""
    specs = [SPECS[0], SPECS[1], SPECS[3]]
    probs = [_req(s) for s in specs]
    prm = pkg.params("svrem", alpha=ALPHA, eta=eta, beta=BETA)
    epochs = 2 * eta + 1
    S = pkg.Server(1 << 31, max_slots=3, n_streams=2)
    tk = [S.submit(P.geom, P.n_subsets, P.g, P.w, prm, epochs, 910 + i) for i, P in enumerate(probs)]
    S.step(0)
    served = [S.poll(t) for t in tk]
    S.close()
    for i, P in enumerate(probs):
        A = pkg.SystemMatrix(P.geom, P.n_subsets)
        R = pkg.Recon(A, P.g, P.w, np.ones((1, P.geom.n_pixels)), prm)
        R.osem_epoch(list(range(P.n_subsets)))
        for o in pkg.splitmix64_orders(910 + i, P.n_subsets, epochs):
            R.svrem_epoch(o)
        assert served[i]["status"] == 0
        np.testing.assert_array_equal(served[i]["f"], R.image().cpu().numpy()[0])
        assert served[i]["phi"] == R.objective()


def test_trim_drops_idle_matrices_and_kept_blocks():
    """svr_serve_trim: dropping the idle matrices makes the next request of
    that key build its own (no reuse counted) with the same result; trimming
    the kept blocks to 0 leaves nothing cached; bad arguments are rejected."""
    P = _req(SPECS[1])
    prm = pkg.params("svrem", alpha=ALPHA, eta=1, beta=BETA)
    S = pkg.Server(1 << 31, max_slots=2, n_streams=2)
    t = S.submit(P.geom, P.n_subsets, P.g, P.w, prm, EPOCHS, 5)
    S.step(0)
    first = S.poll(t)
    assert S.stats()["cached_bytes"] > 0
    S.trim(drop_matrices=True, keep_bytes=1 << 40)
    st = S.stats()
    assert st["cached_bytes"] > 0 and st["matrix_reuses"] == 0  # the matrix's blocks now kept as blocks
    t = S.submit(P.geom, P.n_subsets, P.g, P.w, prm, EPOCHS, 5)
    S.step(0)
    again = S.poll(t)
    st = S.stats()
    assert st["matrix_reuses"] == 0 and st["block_reuses"] > 0
    np.testing.assert_array_equal(first["f"], again["f"])
    S.trim(drop_matrices=True, keep_bytes=0)
    assert S.stats()["cached_bytes"] == 0
    with pytest.raises(pkg.binding.SvrError):
        S.trim(drop_matrices=True, keep_bytes=-1)
    S.close()


def test_storage_types_batch_apart_past_sixty_four_batches():
    """517 resident requests of one tiny geometry (two subsets, so each epoch
    has an anchor and a plain iteration): 516 with int32 indices (65 batches
    of that storage type) and one with 16-bit indices.  Each
    batch holds one storage type however many batches a type has (a key of
    type * 64 + batch index once put the 16-bit request into the 65th int32
    batch); the two kinds of request end bitwise as each does served alone."""
    P = datagen.make_problem(8, 8, 2.0, 4, 12, 2.0, 2, 1e3, seed=77)
    prm = pkg.params("svrem", alpha=ALPHA, eta=1, beta=BETA)
    i32 = pkg.SVR_W_F32 | pkg.binding.SVR_W_INDEX32
    kinds = [i32] * 516 + [pkg.SVR_W_F32]
    S = pkg.Server(4 << 30, max_slots=600, n_streams=3)
    tk = [S.submit(P.geom, 2, P.g, P.w, prm, 2, 900 + i, wtype=wt) for i, wt in enumerate(kinds)]
    S.step(1)
    assert S.stats()["admitted"] == len(kinds) and S.stats()["resident"] == len(kinds)
    S.step(0)
    res = {i: S.poll(tk[i]) for i in (0, 515, 516)}
    S.close()
    for i, r in res.items():
        A = pkg.Server(1 << 30, max_slots=1, n_streams=1)
        t = A.submit(P.geom, 2, P.g, P.w, prm, 2, 900 + i, wtype=kinds[i])
        A.step(0)
        alone = A.poll(t)
        A.close()
        assert r["status"] == 0 and alone["status"] == 0
        np.testing.assert_array_equal(r["f"], alone["f"])
        assert r["phi"] == alone["phi"]
