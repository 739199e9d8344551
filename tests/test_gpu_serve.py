"""Continuous-batching server: results match a run alone and the rollout."""
import time

import numpy as np
import pytest

import wm_synth as S
from oracle import wm_oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def drain(wm, srv, ids, shape, timeout=120.0):
    out, stats = {}, {}
    t0 = time.time()
    while len(out) < len(ids):
        for rid in ids:
            if rid in out:
                continue
            buf = np.empty(shape, np.float32)
            ok, st = wm.wm_serve_poll(srv, rid, buf)
            if ok:
                out[rid], stats[rid] = buf, st
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.002)
    return out, stats


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2503_22235_amd as wm
    assert torch.cuda.is_available()
    ctx = wm.wm_ctx_create(0)
    g = S.Grid(Z=4, Y=9, X=16, C=128, heads=4, Kz=3, Ky=5, Kx=5)
    p6p = S.processor_params(g, 2, seed=1, proc=0)
    p1p = S.processor_params(g, 2, seed=2, proc=1)
    yield wm, torch, ctx, g, p6p, p1p
    ctx.close()


@pytest.mark.parametrize("prec,bf16_state", [(0, False), (1, True)])
def test_serve_alone_equals_mix(env, prec, bf16_state):
    wm, torch, ctx, g, p6p, p1p = env
    p6 = wm.wm_processor_create(ctx, g, 2, 4, prec, p6p)
    p1 = wm.wm_processor_create(ctx, g, 2, 4, prec, p1p)
    shape = (g.Z, g.Y, g.X, g.C)
    rng = np.random.default_rng(3)
    leads = [int(v) for v in rng.integers(0, 20, size=10)] + [0, 13]
    states = S.latent_state(g, len(leads), seed=0)
    say("serve mix", prec, bf16_state, leads)
    mix = wm.wm_serve_create(ctx, p6, p1, max_batch=4, state_bf16=bf16_state, max_slots=6)
    ids = [wm.wm_serve_submit(mix, states[i], leads[i]) for i in range(len(leads))]
    assert wm.wm_serve_status(mix)["slots"] == 6
    res_mix, st_mix = drain(wm, mix, ids, shape)
    mix.close()
    alone = wm.wm_serve_create(ctx, p6, p1, max_batch=1, state_bf16=bf16_state, max_slots=1)
    for i, lead in enumerate(leads):
        rid = wm.wm_serve_submit(alone, states[i], lead)
        r, st = drain(wm, alone, [rid], shape)
        assert np.array_equal(r[rid], res_mix[ids[i]]), f"request {i} differs alone vs in the mix"
        assert st[rid]["steps"] == len(O.schedule(lead))
    alone.close()
    # continuous batching: twelve requests submitted at once with four
    # admitted slots per batch -- some step launch held two or more of them
    cob = max(s["max_cobatch"] for s in st_mix.values())
    say("serve mix: most requests in one step launch", cob)
    assert cob >= 2
    for s in st_mix.values():
        assert s["max_cobatch"] <= 4 and (s["steps"] == 0) == (s["max_cobatch"] == 0)
    for i, rid in enumerate(ids):
        s = st_mix[rid]
        assert s["t_submit"] <= s["t_admit"] <= s["t_done"]
        assert s["lead_hours"] == leads[i]
    if not bf16_state:
        # float32 slots: the served state equals a direct rollout bit for bit
        for i in (0, 3, 11):
            xd = torch.from_numpy(states[i:i + 1].copy()).cuda()
            wm.wm_rollout(ctx, p6, p1, 1, xd, leads[i])
            assert np.array_equal(xd.cpu().numpy()[0], res_mix[ids[i]])
    p6.close()
    p1.close()


@pytest.mark.parametrize("prec,bf16_state", [(1, False), (2, False), (1, True)])
def test_serve_graph_replays_equal_eager(env, prec, bf16_state):
    """cfg.graphs: each (processor, batch size) step runs eagerly once, is
    then captured into a HIP graph and replayed for every later batch of that
    shape, with the server's own eager work (pointer writes or conversions,
    copies, event polls) between replays.  Every result must equal the
    server without graphs bit for bit, and (float32 slots) a direct rollout."""
    wm, torch, ctx, g, p6p, p1p = env
    p6 = wm.wm_processor_create(ctx, g, 2, 4, prec, p6p)
    p1 = wm.wm_processor_create(ctx, g, 2, 4, prec, p1p)
    shape = (g.Z, g.Y, g.X, g.C)
    rng = np.random.default_rng(5)
    leads = [int(v) for v in rng.integers(1, 40, size=12)]
    states = S.latent_state(g, len(leads), seed=2)
    res = {}
    for graphs in (False, True):
        say("serve graphs", graphs, prec, bf16_state, leads)
        srv = wm.wm_serve_create(ctx, p6, p1, max_batch=3, state_bf16=bf16_state, max_slots=5, graphs=graphs)
        ids = [wm.wm_serve_submit(srv, states[i], leads[i]) for i in range(len(leads))]
        out, st = drain(wm, srv, ids, shape)
        srv.close()
        res[graphs] = [out[r] for r in ids]
        assert sum(s["steps"] for s in st.values()) == sum(len(O.schedule(l)) for l in leads)
    for i in range(len(leads)):
        assert np.array_equal(res[True][i], res[False][i]), f"request {i}: graph replay differs from eager"
    if not bf16_state:
        for i in (0, 5, 11):
            xd = torch.from_numpy(states[i:i + 1].copy()).cuda()
            wm.wm_rollout(ctx, p6, p1, 1, xd, leads[i])
            assert np.array_equal(xd.cpu().numpy()[0], res[True][i])
    p6.close()
    p1.close()


def test_serve_result_against_oracle(env):
    wm, torch, ctx, g, p6p, p1p = env
    p6 = wm.wm_processor_create(ctx, g, 2, 4, 1, p6p)
    p1 = wm.wm_processor_create(ctx, g, 2, 4, 1, p1p)
    b6 = [S.split_block_params(g, p6p, b) for b in range(2)]
    b1 = [S.split_block_params(g, p1p, b) for b in range(2)]
    srv = wm.wm_serve_create(ctx, p6, p1, max_batch=2, state_bf16=True)
    x = S.latent_state(g, 1, seed=5)[0]
    rid = wm.wm_serve_submit(srv, x, 8)
    out, _ = drain(wm, srv, [rid], x.shape)
    ref = O.rollout(x, b6, b1, g, 8)
    err = O.rel_l2(out[rid], ref)
    say("serve bf16 lead 8 rel_l2", err)
    assert err < 2e-2
    with pytest.raises(wm.WmError):
        wm.wm_serve_poll(srv, rid)            # already collected
    srv.close()
    p6.close()
    p1.close()


def test_serve_host_forced_limits(env):
    """Limits forced from the host: a budget below one slot, a two-slot budget
    that makes requests wait, unknown ids and invalid configurations."""
    wm, torch, ctx, g, p6p, p1p = env
    p6 = wm.wm_processor_create(ctx, g, 2, 4, 0, p6p)
    p1 = wm.wm_processor_create(ctx, g, 2, 4, 0, p1p)
    shape = (g.Z, g.Y, g.X, g.C)
    slot_bytes = (g.Z * g.Y * g.X * g.C * 4 + 255) // 256 * 256
    say("serve limits: slot", slot_bytes, "bytes")
    # a budget that holds no slot is refused at creation
    with pytest.raises(wm.WmError) as ei:
        wm.wm_serve_create(ctx, p6, p1, max_batch=2, state_bf16=False, hbm_budget_bytes=slot_bytes - 1)
    assert ei.value.code == -2
    # invalid configurations
    for kw in (dict(max_batch=0), dict(max_batch=65), dict(max_slots=-1), dict(max_slots=1025)):
        with pytest.raises(wm.WmError) as ei:
            wm.wm_serve_create(ctx, p6, p1, state_bf16=False, **kw)
        assert ei.value.code == -1, kw
    g2 = S.Grid(Z=4, Y=9, X=16, C=128, heads=4, Kz=3, Ky=3, Kx=5)
    q1 = wm.wm_processor_create(ctx, g2, 2, 4, 0, S.processor_params(g2, 2, seed=2, proc=1))
    with pytest.raises(wm.WmError) as ei:
        wm.wm_serve_create(ctx, p6, q1, state_bf16=False)
    assert ei.value.code == -1
    q1.close()
    # a budget of exactly two slots: requests wait for a slot, results do not change
    srv = wm.wm_serve_create(ctx, p6, p1, max_batch=4, state_bf16=False, hbm_budget_bytes=2 * slot_bytes)
    assert wm.wm_serve_status(srv)["slots"] == 2
    leads = [12, 7, 0, 13, 6, 1, 18, 5]
    states = S.latent_state(g, len(leads), seed=9)
    ids = [wm.wm_serve_submit(srv, states[i], leads[i]) for i in range(len(leads))]
    with pytest.raises(wm.WmError) as ei:
        wm.wm_serve_submit(srv, states[0], -1)
    assert ei.value.code == -1
    with pytest.raises(wm.WmError) as ei:
        wm.wm_serve_poll(srv, max(ids) + 1000)
    assert ei.value.code == -5
    res, st = drain(wm, srv, ids, shape)
    srv.close()
    # slot occupancy: a slot is held from before t_admit until t_done
    events = sorted([(st[r]["t_admit"], 1) for r in ids] + [(st[r]["t_done"], -1) for r in ids],
                    key=lambda e: (e[0], e[1]))
    held = peak = 0
    for _, d in events:
        held += d
        peak = max(peak, held)
    say("serve limits: peak slots held", peak)
    assert peak <= 2
    for i, rid in enumerate(ids):
        xd = torch.from_numpy(states[i:i + 1].copy()).cuda()
        wm.wm_rollout(ctx, p6, p1, 1, xd, leads[i])
        assert np.array_equal(xd.cpu().numpy()[0], res[rid]), f"request {i} (lead {leads[i]})"
        assert st[rid]["steps"] == len(O.schedule(leads[i]))
    p6.close()
    p1.close()
