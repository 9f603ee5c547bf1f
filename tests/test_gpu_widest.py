"""GPU parity of widest-path graphs (APSP_WIDEST): capacities in, widths out.

Every state is compared bit for bit with the oracle's (max, min)
Floyd-Warshall of the capacity matrix: cold starts over several 128-wide
tiles with ragged tails, ties, zero capacities and capacities up to the top
of the range; sequences of every update kind (add, remove, capacity raised
and lowered, an edge deleted and one inserted) on directed and undirected
graphs; queries return the width and a simple path whose smallest capacity
is that width; the adjacency reads back as capacities; the warm start from a
known width matrix, a batch of widest graphs and the no-allocation edge
update give the same matrices as the oracle and the single calls.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2412_15122_amd import workloads as W

pytestmark = pytest.mark.gpu

INF = W.INF
TOP = O.WIDEST_TOP


def log(*a):
    print(*a, flush=True)


def caps(n, cmax, *, undirected, density, seed, zero=0.0):
    return W.random_graph(n, 1, cmax, undirected=undirected, density=density, seed=seed, zero_frac=zero)


def expect(g, C, ids, what):
    assert g.ids() == ids, what
    ref = O.widest_apsp(C)
    got = g.matrix()
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        i, j = bad[0]
        raise AssertionError(f"{what}: {len(bad)} entries differ, first ({ids[i]},{ids[j]}): gpu {got[i, j]} "
                             f"oracle {ref[i, j]}")
    Cd = C.copy()
    np.fill_diagonal(Cd, TOP)
    assert np.array_equal(g.adjacency(), Cd), what
    return ref


def check_paths(g, C, ids, Wm, rng, count=8):
    n = len(ids)
    for _ in range(count):
        a, b = (int(x) for x in rng.integers(0, n, size=2))
        width, path = g.query(ids[a], ids[b])
        assert width == int(Wm[a, b]), (a, b)
        if Wm[a, b] >= INF:
            assert path == []
            continue
        pos = [ids.index(x) for x in path]
        assert pos[0] == a and pos[-1] == b and len(set(pos)) == len(pos)
        assert all(C[x, y] < INF for x, y in zip(pos, pos[1:]))
        assert min((int(C[x, y]) for x, y in zip(pos, pos[1:])), default=TOP) == Wm[a, b], (a, b)


@pytest.mark.parametrize("undirected", [False, True])
def test_widest_cold(undirected):
    from paper_2412_15122_amd.apsp import Graph
    rng = np.random.default_rng(41 + undirected)
    for n, cmax, dens, zero in ((1, 5, 1.0, 0.0), (17, 3, 0.5, 0.2), (129, 10000, 1.0, 0.0),
                                (143, 4, 0.1, 0.1), (300, TOP, 0.05, 0.0), (257, 50, 0.02, 0.0)):
        log("widest cold", n, cmax, dens, zero, undirected)
        C = caps(n, cmax, undirected=undirected, density=dens, seed=int(rng.integers(1 << 30)), zero=zero)
        g = Graph(C, undirected=undirected, capacity=n + 5, widest=True)
        Wm = expect(g, C, list(range(n)), f"cold n={n}")
        check_paths(g, C, list(range(n)), Wm, rng)
        g.close()


@pytest.mark.parametrize("undirected", [False, True])
def test_widest_update_sequences(undirected):
    from paper_2412_15122_amd.apsp import Graph
    rng = np.random.default_rng(51 + undirected)
    n, cmax, dens = 150, 40, 0.35
    C = caps(n, cmax, undirected=undirected, density=dens, seed=int(rng.integers(1 << 30)))
    g = Graph(C, undirected=undirected, capacity=n + 12, widest=True)
    st = W.GraphState(C, undirected)
    ids = list(range(n))
    kinds = [W.REMOVE, W.ADD, W.DECREASE, W.INCREASE, W.DELETE, W.INSERT] * 4
    for t, kind in enumerate(kinds):
        up = W.make_update(rng, st, kind, wmin=1, wmax=cmax, inc_max=2 * cmax, density=dens)
        if up.kind == W.ADD:
            nid = g.add_node(up.w_out, up.w_in)
            C, ids = O.apply_update(C, ids, "add", w_out=up.w_out, w_in=up.w_in, undirected=undirected)
            assert nid == ids[-1]
        elif up.kind == W.REMOVE:
            g.remove_node(up.u)
            C, ids = O.apply_update(C, ids, "remove", u=up.u, undirected=undirected)
        else:
            g.update_edge(up.u, up.v, up.w)
            C, ids = O.apply_update(C, ids, "edge", u=up.u, v=up.v, w=up.w, undirected=undirected)
        Wm = expect(g, C, ids, f"step {t} {up.kind}")
        if t % 4 == 3:
            check_paths(g, C, ids, Wm, rng, count=4)
    g.close()


def test_widest_import_and_noalloc():
    from paper_2412_15122_amd import _native as N
    from paper_2412_15122_amd.apsp import Graph
    rng = np.random.default_rng(61)
    n = 140
    C = caps(n, 25, undirected=False, density=0.5, seed=7)
    Wm = O.widest_apsp(C)
    for exact in (False, True):
        g = Graph.from_matrix(C, Wm, capacity=n + 4, widest=True, exact=exact)
        expect(g, C, list(range(n)), f"import exact={exact}")
        g.close()
    bad = Wm.copy()
    bad[3, 5] = max(0, int(bad[3, 5]) - 1) if bad[3, 5] < INF else 1
    with pytest.raises(N.ApspError):
        Graph.from_matrix(C, bad, capacity=n, widest=True, exact=True)
    # the no-allocation edge update on a widest graph equals the usual one
    g = Graph(C, capacity=n + 4, widest=True)
    h = g.clone()
    ids = list(range(n))
    for t in range(12):
        u, v = (int(x) for x in rng.choice(n, size=2, replace=False))
        c = int(rng.integers(0, 40)) if t % 4 else INF
        g.update_edge_noalloc(u, v, c)
        h.update_edge(u, v, c)
        C, ids = O.apply_update(C, ids, "edge", u=u, v=v, w=c)
        assert np.array_equal(g.matrix(), h.matrix()), t
    expect(g, C, ids, "noalloc")
    g.close()
    h.close()


@pytest.mark.parametrize("config", [{"use_graph": False, "variant": 1}, {"use_graph": True, "variant": 3}])
def test_widest_batch(config):
    """Widest graphs in one batched launch (the minimax kernels over stored
    capacities): matrices, ids and query widths equal the single calls and
    the oracle."""
    import torch
    from paper_2412_15122_amd.apsp import Graph
    from paper_2412_15122_amd.batch import Batch
    rng = np.random.default_rng(71 + config["variant"])
    sizes = [3, 40, 143, 300, 129]
    ga, states, per = [], [], []
    for gi, n in enumerate(sizes):
        und = gi % 2 == 1
        C = caps(n, 30, undirected=und, density=0.4, seed=800 + gi)
        ga.append(Graph(C, undirected=und, capacity=n + 8, widest=True))
        st = W.GraphState(C, und)
        seq = []
        for t in range(6):
            k = [W.ADD, W.REMOVE, W.DECREASE, W.INCREASE, W.DELETE, W.INSERT][int(rng.integers(6))]
            if k == W.REMOVE and len(st.live) < 3:
                k = W.ADD
            try:
                up = W.make_update(rng, st, k, wmin=1, wmax=30, inc_max=60, density=0.4)
            except RuntimeError:  # no present (or absent) edge left between live nodes
                up = W.make_update(rng, st, W.ADD, wmin=1, wmax=30, inc_max=60, density=0.4)
            if up.kind == W.ADD:
                seq.append(("add", gi, up.w_out, up.w_in))
            elif up.kind == W.REMOVE:
                seq.append(("remove", gi, up.u))
            else:
                seq.append(("edge", gi, up.u, up.v, up.w))
            if len(st.live) >= 2 and t % 2 == 1:
                a, c = rng.choice(len(st.live), size=2, replace=False)
                seq.append(("query", gi, st.live[int(a)], st.live[int(c)]))
        states.append(st)
        per.append(seq)
    items = [it for t in range(max(map(len, per))) for seq in per if t < len(seq) for it in [seq[t]]]
    gb = [g.clone() for g in ga]
    b = Batch(len(ga), len(items), **config)
    res = b.run(ga, items)
    b.status()
    torch.cuda.synchronize()
    answers = {}
    for t, it in enumerate(items):
        g = gb[it[1]]
        if it[0] == "add":
            g.add_node(it[2], None if g.undirected else it[3])
        elif it[0] == "remove":
            g.remove_node(it[2])
        elif it[0] == "edge":
            g.update_edge(it[2], it[3], it[4])
        else:
            answers[t] = g.query(it[2], it[3])[0]
    for gi in range(len(ga)):
        assert ga[gi].ids() == gb[gi].ids() == states[gi].live
        assert torch.equal(ga[gi].matrix_device("D"), gb[gi].matrix_device("D")), gi
        assert np.array_equal(ga[gi].matrix(), O.widest_apsp(states[gi].dense())), gi
    for t, width in answers.items():
        assert res[t].get()[0] == width, t
    b.close()
    for g in ga + gb:
        g.close()
