"""Batched and served reconstructions on the GPU.

A slice's arithmetic never depends on the batch or the served mix it runs in, so every
batched or served result must equal the one vp_reconstruct returns for that slice alone,
bit for bit; the solo results themselves are checked against the oracle elsewhere.
"""

import numpy as np
import pytest

import oracle as O
from synth import configs

pytestmark = pytest.mark.gpu

CASES = [
    dict(n=48, n_spec=6, n_blades=4, lines=12),
    dict(n=40, n_spec=5, n_time=3, n_blades=6, lines=8),
    dict(n=80, n_spec=5, n_blades=3, lines=10, f=3.0),
    dict(n=60, n_spec=3, n_blades=5, lines=7),
    dict(n=64, n_spec=8, n_time=4, n_blades=10, lines=12, seed=11),
]


def _problems(B, steps):
    out = []
    for kw, st in zip(CASES, steps):
        case = configs.small_case(**kw)
        plan = B.Plan.from_geometry(case.geometry())
        y = O.simulate_measurements(case)
        out.append((case, plan, y, B.vp_options_default(n_steps=st)))
    return out


def _same(a, b):
    return (np.array_equal(a["vol"], b["vol"]) and np.array_equal(a["proj"], b["proj"])
            and np.array_equal(a["water"], b["water"]) and np.array_equal(a["fat"], b["fat"])
            and a["final_loss"] == b["final_loss"])


def test_served_results_equal_solo_results(gpu_lib):
    from paper_2311_13177_amd import binding as B

    probs = _problems(B, [9, 17, 4, 12, 23])
    solo = [B.vp_reconstruct(p, y, o) for _, p, y, o in probs]
    srv = B.Server(hbm_budget=4 << 30, max_slots=8)
    ids = [srv.submit(p, y, o) for _, p, y, o in probs]
    got = [srv.wait(i) for i in ids]
    for g, s, (_, _, _, o) in zip(got, solo, probs):
        assert g["status"] == 0 and g["steps_done"] == o.n_steps
        assert _same(g, s)
    st = srv.stats()
    assert st["completed"] == len(probs) and st["p99_us"] >= st["p50_us"] > 0 and st["throughput_rps"] > 0
    srv.close()


def test_small_budget_queues_and_still_matches(gpu_lib):
    from paper_2311_13177_amd import binding as B

    probs = _problems(B, [6, 7, 5])
    need = max(p.device_bytes(o) for _, p, _, o in probs)
    srv = B.Server(hbm_budget=need, max_slots=8)
    ids = [srv.submit(p, y, o) for _, p, y, o in probs]
    # requests arriving while others run are admitted as memory frees up
    late = _problems(B, [0, 0, 0, 8])[3]
    ids.append(srv.submit(late[1], late[2], late[3]))
    got = [srv.wait(i) for i in ids]
    for g, (_, p, y, o) in zip(got, probs + [late]):
        assert _same(g, B.vp_reconstruct(p, y, o))
    # collected out of order: the finished first request is moved to host to make room
    a = srv.submit(probs[0][1], probs[0][2], probs[0][3])
    b = srv.submit(probs[1][1], probs[1][2], probs[1][3])
    gb = srv.wait(b)
    ga = srv.wait(a)
    assert _same(ga, B.vp_reconstruct(probs[0][1], probs[0][2], probs[0][3]))
    assert _same(gb, B.vp_reconstruct(probs[1][1], probs[1][2], probs[1][3]))
    srv.close()


def test_server_errors_and_cancel(gpu_lib):
    from paper_2311_13177_amd import binding as B

    (_, plan, y, opts), = _problems(B, [40])[:1]
    srv = B.Server(hbm_budget=plan.device_bytes(opts), max_slots=1)
    tiny = B.Server(hbm_budget=1024, max_slots=1)
    with pytest.raises(B.VPError) as ei:
        tiny.submit(plan, y, opts)
    assert ei.value.status == B.VP_ERR_BUDGET
    tiny.close()
    bad = y.copy()
    bad[0, 0, 1] = np.inf
    with pytest.raises(B.VPError) as ei:
        srv.submit(plan, bad, opts)
    assert ei.value.status == B.VP_ERR_NONFINITE
    first = srv.submit(plan, y, B.vp_options_default(n_steps=400))
    queued = srv.submit(plan, y, opts)     # the budget holds one request: this one waits
    srv.cancel(queued)
    r = srv.wait(queued, raise_on_error=False)
    assert r["status"] == B.VP_ERR_CANCELLED
    srv.cancel(first)
    r = srv.wait(first, raise_on_error=False)
    assert r["status"] in (B.VP_ERR_CANCELLED, B.VP_OK)
    with pytest.raises(B.VPError) as ei:
        srv.poll(first)
    assert ei.value.status == B.VP_ERR_NOT_FOUND
    srv.close()


def test_resident_batch_in_parts_equals_solo(gpu_lib):
    # a resident batch stepped in parts (graph replays, eager stage-timed steps, more graph
    # replays) reaches each slice's own step count and equals its solo fit bit for bit;
    # slices that stop earlier stay where they stopped
    from paper_2311_13177_amd import binding as B

    probs = _problems(B, [5, 9, 7, 9, 3])
    solo = [B.vp_reconstruct(p, y, o) for _, p, y, o in probs]
    batch = B.Batch([p for _, p, _, _ in probs], [y for _, _, y, _ in probs], [o for _, _, _, o in probs])
    batch.step(3, use_graph=True)
    st = batch.stage_times(2)
    assert tuple(st) == B.Batch.STAGES and all(v > 0 for v in st.values())
    batch.step(4, use_graph=True)
    for i, (s, (_, _, _, o)) in enumerate(zip(solo, probs)):
        r = batch.read(i)
        assert r["status"] == 0 and r["steps_done"] == min(o.n_steps, 9)
        if o.n_steps <= 9:
            assert _same(r, s)
    batch.close()


def _workload(B, case, **overrides):
    plan = B.Plan.from_geometry(case.geometry())
    y = O.simulate_measurements(case)
    opts = B.vp_options_default(n_steps=case.n_steps, tv_weight=case.tv_weight, lr=case.lr, **overrides)
    return plan, y, opts


def test_batched_slice_matches_the_oracle_fit(gpu_lib):
    """Slice 3 of the 64-slice batch (128^2, S 16, 16 blades, 200 Adam steps), fitted in a
    batch beside slice 6, against the FP64 oracle's fit of that slice stored by
    tests/golden/make_converged.py (render and objective, at twice the oracle's own spread
    or 1e-3)."""
    from parity import check_converged
    from paper_2311_13177_amd import binding as B

    probs = [_workload(B, configs.batch_slice(j), autotune=1) for j in (3, 6)]
    got = B.vp_batch_reconstruct([p for p, _, _ in probs], [y for _, y, _ in probs], [o for _, _, o in probs])
    assert got[0]["status"] == 0 and got[0]["steps_done"] == 200
    r = check_converged("batch_3", got[0]["proj"], got[0]["final_loss"])
    print("batch_3", r)


def test_served_requests_match_the_oracle_fits(gpu_lib):
    """Two requests of the served stream at their own sizes and full step counts, a static
    one (request 17: 128^2, S 16, 16 blades, 200 steps) and a dynamic one (request 4:
    128^2, S 16, T 8, 24 blades, 800 steps), served together with a third request, against
    the FP64 oracle's fits stored by tests/golden/make_converged.py."""
    from parity import check_converged
    from paper_2311_13177_amd import binding as B

    names = {17: "serve_17", 4: "serve_4"}
    probs = {i: _workload(B, configs.serving_request(i)) for i in (17, 4, 9)}
    srv = B.Server(hbm_budget=8 << 30, max_slots=4)
    ids = {i: srv.submit(p, y, o) for i, (p, y, o) in probs.items()}
    got = {i: srv.wait(rid, volume=False) for i, rid in ids.items()}
    srv.close()
    for i, name in names.items():
        assert got[i]["status"] == 0 and got[i]["steps_done"] == probs[i][2].n_steps
        r = check_converged(name, got[i]["proj"], got[i]["final_loss"])
        print(name, r)


def test_streamed_batch_equals_cached_solo(gpu_lib):
    """A step whose state (both volume copies and the Adam moments) exceeds the 256 MiB
    Infinity Cache streams its update: the moment loads, the update's stores and the
    previous knot's plane loads carry the non-temporal cache hint. That changes no result.
    The batch of a 192^2 x 32 x 16 slice (604 MB of state) and a 64^2 slice streams, the
    64^2 slice alone (4 MB) does not, and its results must agree bit for bit, with the
    batch in its own tile shape, in the phased gather and with the separate update pass
    (each kernel's streamed variant)."""
    from paper_2311_13177_amd import binding as B

    cases = [configs.CONFIGS["dynamic_192"](), configs.CONFIGS["static_64"]()]
    plans = [B.Plan.from_geometry(c.geometry()) for c in cases]
    ys = [O.simulate_measurements(c) for c in cases]
    steps = [12, 9]
    solo = [B.vp_reconstruct(p, y, B.vp_options_default(n_steps=st)) for p, y, st in zip(plans, ys, steps)]
    for tiles in (None, (2, 2, 4, 2, 0, 8, 8, 0), (4, 1, 4, 4, 4, 8, 8, 0)):
        extra = {} if tiles is None else dict(tiles=tiles)
        opts = [B.vp_options_default(n_steps=st, **extra) for st in steps]
        got = B.vp_batch_reconstruct(plans, ys, opts)
        for g, s in zip(got, solo):
            assert g["status"] == 0 and _same(g, s), tiles
