"""Seeded input generators: determinism, value ranges and stream bookkeeping."""
import numpy as np

from paper_2412_15122_amd import workloads as W

INF = W.INF


def test_random_graph_shapes_and_ranges():
    a = W.random_graph(50, 1, 1000, seed=1)
    assert a.dtype == np.int32 and a.shape == (50, 50)
    assert np.all(np.diag(a) == 0)
    off = a[~np.eye(50, dtype=bool)]
    assert off.min() >= 1 and off.max() <= 1000
    b = W.random_graph(50, 1, 1000, seed=1)
    assert np.array_equal(a, b)
    u = W.random_graph(40, 1, 9, undirected=True, density=0.5, seed=2)
    assert np.array_equal(u, u.T)
    assert np.any(u == INF)
    s = W.symmetric_complete_graph(33, 1, 10000, 5)
    assert np.array_equal(s, s.T) and np.all(np.diag(s) == 0) and s[s > 0].min() >= 1


def test_config1_stream():
    wl = W.config1()
    kinds = [u.kind for u in wl.updates]
    assert kinds == [W.ADD, W.REMOVE, W.DECREASE, W.INCREASE]
    add = wl.updates[0]
    assert add.new_id == 256 and add.w_out.shape == (256,) and add.w_in.shape == (256,)
    assert 1 <= add.w_out.min() and add.w_out.max() <= 1000
    dec, inc = wl.updates[2], wl.updates[3]
    assert 1 <= dec.w <= dec.old
    assert inc.old <= inc.w <= max(inc.old, 2000)
    again = W.config1()
    assert [(u.kind, u.u, u.v, u.w) for u in again.updates] == [(u.kind, u.u, u.v, u.w) for u in wl.updates]


def test_config3_block_counts():
    adj = W.symmetric_complete_graph(64, 1, 10000, 3)
    st = W.Config3Stream(adj, seed=9)
    worst = W.lightest_edges(adj, 1, True)[0]
    block = st.next_block(worst=(worst[0], worst[1], 20000))
    assert len(block) == 1000
    counts = {k: sum(1 for u in block if u.kind == k) for k in (W.ADD, W.REMOVE, W.DECREASE, W.INCREASE)}
    assert counts == W.CFG3_COUNTS
    assert block[0].kind == W.INCREASE and (block[0].u, block[0].v) == worst[:2]
    live = set(range(64))
    max_id = 63
    for u in block:
        if u.kind == W.ADD:
            assert u.new_id == max_id + 1
            max_id = u.new_id
            assert np.array_equal(u.w_out, u.w_in)
            live.add(u.new_id)
        elif u.kind == W.REMOVE:
            assert u.u in live
            live.remove(u.u)
        else:
            assert u.u in live and u.v in live and u.u != u.v
    assert live == set(st.state.live)


def test_graph_state_weights_track_updates():
    adj = W.random_graph(5, 1, 9, seed=4)
    st = W.GraphState(adj, False)
    nid = st.add(np.array([1, 2, 3, 4, 5], np.int32), np.array([6, 7, 8, 9, 10], np.int32))
    nid2 = st.add(np.arange(11, 17, dtype=np.int32), np.arange(21, 27, dtype=np.int32))
    assert st.weight(nid, 2) == 3 and st.weight(2, nid) == 8
    assert st.weight(nid2, nid) == 16 and st.weight(nid, nid2) == 26
    st.set_weight(nid, nid2, 99)
    assert st.weight(nid, nid2) == 99
    st.remove(3)
    assert 3 not in st.live
    d = st.dense()
    assert d.shape == (6, 6) and np.all(np.diag(d) == 0)


def test_lightest_edges():
    a = W.random_graph(30, 1, 100, seed=8)
    got = W.lightest_edges(a, 10, False)
    ws = sorted((int(a[u, v]), u, v) for u in range(30) for v in range(30) if u != v)[:10]
    assert [(w, u, v) for (u, v, w) in got] == ws


def test_config4_and_5_shapes():
    gs = W.config4(graphs=6, updates_per_graph=8)
    assert len(gs) == 6
    for g in gs:
        assert 128 <= g.adj.shape[0] <= 2048 and len(g.updates) == 8
    adjs = W.config5_graphs(graphs=3, nmin=16, nmax=40)
    req = W.Config5Requests(adjs, seed=1)
    t = req.arrivals(1000.0, 100)
    assert np.all(np.diff(t) > 0)
    for _ in range(50):
        g, kind, payload = req.next_request()
        assert 0 <= g < 3
