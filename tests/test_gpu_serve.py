"""Serving loop: requests admitted by HBM footprint into a running batch give
the same result as when run alone (bitwise: per-domain arithmetic does not
depend on the batch), and the budget is never exceeded."""
import numpy as np
import pytest

from paper_1909_04153_amd import scenarios as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1909_04153_amd import bq, serve

    bq.load()
    return bq, serve


def _specs():
    ends = [0.6, 0.3, 30.0, 0.45]
    out = [S.sloping_beach(nx=192, ny=64, dx=0.1, x_toe=2.0),
           S.solitary_flat(nx=160, ny=48, x0=2.0),
           S.rip_beach_scaled(96, 64, cfl=0.125, fstar_order=1),
           S.solitary_flat(nx=300, ny=32, x0=3.0)]
    for s, t in zip(out, ends):
        s["params"]["t_end"] = t
    return out


@pytest.mark.parametrize("static_tables", [True, False])
def test_served_results_equal_solo_runs(mods, static_tables):
    bq, serve = mods
    specs = _specs()
    solo = []
    for s in specs:
        d = bq.domain_from_spec(s, precision=bq.FP32)
        i = d.sync()
        while i.status == bq.OK:
            d.step(64)
            i = d.sync()
        assert i.status == bq.EDONE
        solo.append((i.n, [d.read(f) for f in ("eta", "P", "Q")]))
        d.close()
    budget = sum(bq.workspace_bytes(s["params"], bq.FP32) for s in specs[:2]) + 1024
    srv = serve.Server(budget, max_slots=3, precision=bq.FP32, chunk_steps=8, keep_results=True,
                       static_tables=static_tables)
    reqs = [serve.Request(k, s, arrival=0.02 * k) for k, s in enumerate(specs)]
    stats = srv.run(reqs, max_wall=120.0)
    assert srv.peak_used <= budget
    for r, (n, ref) in zip(stats.requests, solo):
        assert r.status == bq.EDONE and r.steps == n, (r.rid, r.status, r.steps, n)
        for f, x in zip(("eta", "P", "Q"), ref):
            assert np.array_equal(r.result[f], x), (r.rid, f)
    summ = stats.summary()
    assert summ["completed"] == len(specs) and summ["p99_s"] >= summ["p50_s"] > 0


def test_batch_status_matches_member_sync(mods):
    # one readback for the whole batch gives each member's status, step
    # count and time as its own bq_sync does, including a member that
    # reached t_end (EDONE) while the others continue
    bq, _ = mods
    specs = _specs()
    specs[1]["params"]["t_end"] = 0.05
    for k in (0, 3):
        specs[k]["params"]["t_end"] = 30.0
    doms = [bq.domain_from_spec(s, precision=bq.FP32) for s in specs]
    b = bq.Batch(doms)
    for static in (False, True):
        b.set(doms, static=static)
        b.step(40)
        st, n, t = b.status()
        for k, d in enumerate(doms):
            i = d.sync()
            assert (st[k], n[k], t[k]) == (i.status, i.n, i.t), (static, k)
        assert st[1] == bq.EDONE and all(st[k] == bq.OK for k in (0, 2, 3))
    b.close()
