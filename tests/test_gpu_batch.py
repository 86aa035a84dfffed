"""The persistent work-queue path: identical to per-iteration launches and to
single registrations (bitwise), per-problem statuses, and oracle parity of a
batch of uneven problems."""
import numpy as np
import pytest

import synth
from oracle import covariance as oc
from oracle import gicp as og
from oracle import se3

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def g():
    import paper_2403_12550_amd as g
    g.lib()
    return g


@pytest.fixture(scope="module")
def ctx(g):
    import torch
    torch.cuda.set_device(0)
    c = g.Context(0)
    yield c
    c.close()


def _c1(g, ctx, n=5000, seed=0):
    pr = synth.c1_problem(n=n, room_seed=seed, src_seed=seed + 1, tgt_seed=seed + 2, tf_seed=seed + 3)
    src, tgt = g.to_soa(pr.src), g.to_soa(pr.tgt)
    tcov = ctx.covariances(tgt, 20, reg_mode=1)
    gm = ctx.map_build(tgt, tcov, cell=0.1)
    return pr, src, gm


@pytest.mark.parametrize("acc", [0, 1, 2])
def test_three_paths_agree(g, ctx, acc):
    """Batched launches (default), per-registration launches and the work
    queue evaluate the same expressions with the same chunking and summation
    order: they agree bitwise."""
    _say("paths", acc)
    pr, src, gm = _c1(g, ctx)
    a = ctx.register(src, gm, pr.init, g.params(max_it=30, precision=acc))
    b = ctx.register(src, gm, pr.init, g.params(max_it=30, precision=acc, flags=g.FLAG_MULTI_LAUNCH))
    q = ctx.register(src, gm, pr.init, g.params(max_it=30, precision=acc, flags=g.FLAG_QUEUE))
    for r in (a, b, q):
        assert r.status == 0 and r.iters == 30
    for r in (b, q):
        assert (a.pose == r.pose).all() and (a.H == r.H).all() and (a.b == r.b).all()


def test_queue_early_exit_matches(g, ctx):
    _say("queue_early_exit")
    pr, src, gm = _c1(g, ctx)
    prm = dict(max_it=30, conv_rot=1e-6, conv_trans=1e-6)
    a = ctx.register(src, gm, pr.init, g.params(**prm))
    b = ctx.register(src, gm, pr.init, g.params(flags=g.FLAG_MULTI_LAUNCH, **prm))
    q = ctx.register(src, gm, pr.init, g.params(flags=g.FLAG_QUEUE, **prm))
    assert a.converged and b.converged and q.converged and a.iters == b.iters == q.iters < 30
    assert (a.pose == b.pose).all() and (a.pose == q.pose).all()


def _batch_problems(g, ctx, sizes, seed0=5000):
    import torch
    out = []
    for i, (ns, m) in enumerate(sizes):
        rng = np.random.default_rng(seed0 + i)
        room = synth.make_room(seed0 + i)
        tp, tn = synth.sample_surface(room, m, seed0 + i + 1, 0.001)
        sp, _ = synth.sample_surface(room, ns, seed0 + i + 2, 0.002)
        T = synth.random_offset(rng, 3.0, 0.05)
        src = (sp - T[:3, 3]) @ T[:3, :3]
        cov = synth.disc_covariances(tn, seed0 + i + 3)
        means = g.to_soa(tp.astype(np.float32))
        gm = ctx.map_build(means, g.to_soa(cov.astype(np.float32)), cell=0.0, reg_mode=1)
        out.append(dict(src_np=src.astype(np.float32), tgt_np=tp.astype(np.float32), cov_np=cov.astype(np.float32),
                        src=g.to_soa(src.astype(np.float32)), map=gm, T=T))
        torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("flags", [0, 2, 4])
def test_batch_equals_single(g, ctx, flags):
    _say("batch_vs_single", flags)
    sizes = [(2000, 30000), (7000, 60000), (15000, 20000), (300, 50000), (40000, 100000)]
    probs = _batch_problems(g, ctx, sizes)
    prm = g.params(max_it=20, conv_rot=1e-6, conv_trans=1e-6, cell_src=0.0, flags=flags)
    batch = ctx.register_batch([(p["src"], None, p["map"], np.eye(4)) for p in probs], prm)
    for p, rb in zip(probs, batch):
        rs = ctx.register(p["src"], p["map"], np.eye(4), g.params(max_it=20, conv_rot=1e-6, conv_trans=1e-6,
                                                                  flags=g.FLAG_MULTI_LAUNCH))
        assert rb.status == rs.status == 0
        assert rb.iters == rs.iters
        assert (rb.pose == rs.pose).all() and (rb.H == rs.H).all()
    for p in probs:
        p["map"].close()


def test_batch_oracle_parity(g, ctx):
    _say("batch_oracle")
    sizes = [(3000, 40000), (9000, 80000)]
    probs = _batch_problems(g, ctx, sizes, seed0=6000)
    prm = g.params(max_it=20, conv_rot=1e-6, conv_trans=1e-6)
    batch = ctx.register_batch([(p["src"], None, p["map"], np.eye(4)) for p in probs], prm)
    for p, rb in zip(probs, batch):
        cs = oc.covariances(p["src_np"], 20)
        ct = oc.regularise6(p["cov_np"], oc.REG_PLANE, 1e-3)
        o = og.register(p["src_np"], cs, p["tgt_np"], ct, np.eye(4), r_max=0.1, max_it=20,
                        conv_rot=1e-6, conv_trans=1e-6)
        dr, dt = se3.pose_error(rb.pose, o.pose)
        _say(f"  rot {dr:.2e} trans {dt:.2e} it {rb.iters}/{o.iters}")
        assert dr < 1e-5 and dt < 1e-5
        p["map"].close()


def test_batch_statuses(g, ctx):
    _say("batch_statuses")
    pr, src, gm = _c1(g, ctx, n=2000)
    far = np.eye(4)
    far[:3, 3] = [30, 0, 0]
    for flags in (0, 1, 2, 4):
        res = ctx.register_batch([(src, None, gm, np.eye(4)), (src, None, gm, far), (src, None, gm, np.eye(4))],
                                 g.params(max_it=10, flags=flags))
        assert [r.status for r in res] == [0, 3, 0]
        assert res[1].iters == 1 and np.allclose(res[1].pose, far)
        assert (res[0].pose == res[2].pose).all()


def test_batch_arg_errors(g, ctx):
    pr, src, gm = _c1(g, ctx, n=500)
    with pytest.raises(g.GicpError):
        ctx.register_batch([], g.params())
    with pytest.raises(g.GicpError):
        ctx.register_batch([(src, None, gm, np.eye(4))], g.params(r_max=-1.0))


def test_graph_replays_match_launches(g, ctx):
    """The graph-captured iterations replay the default launches bit for bit:
    several calls per batch shape (cached graph, replayed with eager calls of
    other shapes in between), each replay checked."""
    _say("graph_replays")
    sizes = [(2000, 30000), (7000, 60000), (15000, 20000), (300, 50000)]
    probs = _batch_problems(g, ctx, sizes, seed0=7000)
    kw = dict(max_it=20, conv_rot=1e-6, conv_trans=1e-6)
    batches = [probs[:2], probs[1:], probs[:2], [probs[3]], probs[1:], probs[:2]]
    for rnd, bp in enumerate(batches):
        items = [(p["src"], None, p["map"], np.eye(4)) for p in bp]
        ref = ctx.register_batch(items, g.params(**kw))
        got = ctx.register_batch(items, g.params(flags=g.FLAG_GRAPH, **kw))
        for a, b in zip(ref, got):
            assert a.status == b.status == 0 and a.iters == b.iters, rnd
            assert (a.pose == b.pose).all() and (a.H == b.H).all() and (a.b == b.b).all(), rnd
    with pytest.raises(g.GicpError):
        ctx.register_batch([(probs[0]["src"], None, probs[0]["map"], np.eye(4))], g.params(flags=64))
    for p in probs:
        p["map"].close()


def test_autotune_choices(g, ctx, tmp_path, monkeypatch):
    """The autotuner times real library calls and picks a candidate; the
    choice changes speed only (results stay exact for every candidate)."""
    from paper_2403_12550_amd import autotune as at
    monkeypatch.setattr(at, "CACHE", str(tmp_path / "tune.json"))
    _say("autotune")
    pr, src, gm = _c1(g, ctx, n=5000)
    cell, rec = at.tune_source_cell(ctx, src, 20)
    assert cell > 0 and rec["factor"] in at.SRC_FACTORS and len(rec["ms"]) == len(at.SRC_FACTORS)
    # cached on the second call
    cell2, rec2 = at.tune_source_cell(ctx, src, 20)
    assert cell2 == cell and rec2 == rec
    # every candidate gives the same covariances bit for bit
    base = ctx.covariances(src, 20, cell=cell).cpu().numpy()
    for f in at.SRC_FACTORS[:3]:
        other = ctx.covariances(src, 20, cell=ctx.estimate_cell(src, 20) * f).cpu().numpy()
        assert (other.view(np.uint32) == base.view(np.uint32)).all()
    frames = [src] * 8
    b, recb = at.tune_batch(ctx, gm, frames, [np.eye(4)] * 8, g.params(max_it=10), use_cache=False)
    assert b in at.BATCHES and b <= 8
    gm.close()


def test_lanes_per_point_bitwise(g, ctx):
    """The lanes per source point (gicp_params.lanes) change only how a
    point's search is split: every form gives bitwise the same registration
    with 2 and 4 lanes (batched launches, graph replay, work queue,
    per-registration launches, and gicp_track in its slot, launch-pair and
    graph forms); other values are refused."""
    _say("lanes")
    pr, src, gm = _c1(g, ctx)
    ref = ctx.register(src, gm, pr.init, g.params(max_it=12))
    for flags in (0, g.FLAG_GRAPH, g.FLAG_QUEUE, g.FLAG_MULTI_LAUNCH):
        for lanes in (2, 4):
            r = ctx.register(src, gm, pr.init, g.params(max_it=12, flags=flags, lanes=lanes))
            assert (r.pose == ref.pose).all() and (r.H == ref.H).all() and r.iters == ref.iters, (flags, lanes)
    frames = [src, src, src]
    tref = ctx.track(frames, gm, pr.init, prm=g.params(max_it=12, conv_rot=1e-6, conv_trans=1e-6))
    for flags in (0, g.FLAG_MULTI_LAUNCH, g.FLAG_GRAPH):
        for lanes in (2, 4):
            tr = ctx.track(frames, gm, pr.init, prm=g.params(max_it=12, conv_rot=1e-6, conv_trans=1e-6,
                                                             flags=flags, lanes=lanes))
            for a, b in zip(tref, tr):
                assert (a.pose == b.pose).all() and (a.H == b.H).all() and a.iters == b.iters, (flags, lanes)
    for bad in (1, 3, 8, -2):
        with pytest.raises(g.GicpError):
            ctx.register(src, gm, pr.init, g.params(max_it=2, lanes=bad))
    gm.close()


def test_autotune_forms(g, ctx, tmp_path, monkeypatch):
    """The form and lanes tuners time every candidate on real calls, cache
    their choice, and the chosen form gives the default form's results."""
    from paper_2403_12550_amd import autotune as at
    monkeypatch.setattr(at, "CACHE", str(tmp_path / "tune.json"))
    _say("autotune forms")
    pr, src, gm = _c1(g, ctx, n=5000)
    items = [(src, None, gm, pr.init)] * 4
    prm = g.params(max_it=10)
    (flags, lanes), rec = at.tune_form(ctx, items, prm)
    assert (rec["form"], flags, lanes) in [(n, f, ln) for n, f, ln in at.FORMS] and len(rec["ms"]) == len(at.FORMS)
    assert at.tune_form(ctx, items, prm)[1] == rec   # cached
    ref = ctx.register_batch(items, prm)
    got = ctx.register_batch(items, g.params(max_it=10, flags=flags, lanes=lanes))
    for a, b in zip(ref, got):
        assert (a.pose == b.pose).all()
    lanes_t, rect = at.tune_track_lanes(ctx, [src, src], gm, pr.init, 0, prm)
    assert lanes_t in at.TRACK_LANES and len(rect["ms"]) == len(at.TRACK_LANES)
    gm.close()


def test_batch_more_than_one_segment_group(g, ctx):
    """More sources than one segmented grid holds (255): the call splits them
    into groups; every result equals the single registration."""
    _say("batch_300")
    pr, src, gm = _c1(g, ctx, n=1500)
    rng = np.random.default_rng(11)
    inits = []
    for _ in range(300):
        T = np.eye(4)
        T[:3, 3] = rng.normal(0, 0.01, 3)
        inits.append(T)
    prm = g.params(max_it=8)
    batch = ctx.register_batch([(src, None, gm, T) for T in inits], prm)
    for j in (0, 254, 255, 299):
        rs = ctx.register(src, gm, inits[j], prm)
        assert batch[j].status == rs.status == 0
        assert (batch[j].pose == rs.pose).all() and (batch[j].H == rs.H).all(), j
    gm.close()
