"""GPU parity of the device-side setup: the pair distribution built from the
states on the device (Algorithm 2's preprocessing), state-only updates,
VertexDiamUB (Algorithm 1) and the phase outputs of Algorithm 1.

Every value compared here is an integer or a single IEEE operation on exact
integers, so every comparison is exact."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import gpu_context, gpu_hits, oracle_hits, oracle_objects, same_stats

pytestmark = pytest.mark.gpu


def disjoint_union(graphs, directed=False, name="union"):
    src, dst, off = [], [], 0
    for g in graphs:
        s, d = g.edges()
        src.append(s + off)
        dst.append(d + off)
        off += g.n
    return W.csr_from_edges(off, np.concatenate(src), np.concatenate(dst), directed, name=name)


def state_cases():
    rng = np.random.default_rng(42)
    out = []
    g = W.path_graph(2)
    out.append((g, np.array([0, 65535], np.uint16)))
    g = W.er_graph(1000, 5000, 1)
    out.append((g, W.uniform_states(g.n, rng)))
    g = W.er_graph(5001, 20000, 2)          # several radix tiles and a ragged tail
    out.append((g, W.beta_states(g.n, rng)))
    out.append((g, rng.choice(np.array([0, 7, 65535], np.uint16), size=g.n)))   # heavy ties
    out.append((g, W.skewed_states(g.n, rng)))
    out.append(W.with_isolated_component(W.er_graph(300, 700, 9), 50))
    g = W.random_small_graph(80, 0.05, 17, directed=True)
    out.append(W.with_isolated_component(g, 20))
    g = W.rmat_graph(14, 8, seed=3, directed=True)   # nodes without arcs among the active ones
    out.append((g, W.beta_states(g.n, rng)))
    k = np.zeros(g.n, np.uint16)
    k[-1] = 1                                         # one node apart from all others
    out.append((g, k))
    return out


@pytest.mark.parametrize("ci", range(9))
def test_state_build_matches_oracle(ci):
    """The device-built ranks, W, P, S_v, d_v, C and d_hat equal the oracle's
    preprocessing (which the CPU suite pins to brute force) bit for bit;
    P[i] = C - r[i+1] relates the oracle's suffix form to the device's prefix
    form."""
    g, k = state_cases()[ci]
    st = O.States(k)
    a = st.arrays()
    c = gpu_context(g, k)
    d = c.debug_states()
    n = g.n
    assert d["C"] == st.C
    assert np.array_equal(d["perm"][1:], a["perm"][1:n + 1]) and d["perm"][0] == -1
    assert np.array_equal(d["kr"][1:n + 1].astype(np.uint64), a["x"][1:n + 1])
    assert d["kr"][0] == 0 and d["kr"][n + 1] == 0
    assert np.array_equal(d["W"][1:n + 2], a["w"][1:n + 2]) and d["W"][0] == 0
    want_P = np.array([st.C - int(a["r"][i + 1]) for i in range(n + 1)], dtype=np.uint64)
    assert np.array_equal(d["P"], want_P)
    assert np.array_equal(d["S_v"], a["S"])
    want_d = np.where(a["S"] > 0, float(st.C) / np.where(a["S"] > 0, a["S"], 1.0), 0.0)
    assert np.array_equal(d["d_v"], want_d)
    assert d["d_hat"] == max(1.0, float(want_d.max()))
    c.close()


def test_state_only_updates():
    """New states on a loaded graph (host array, device tensor, degenerate,
    then valid again): each set of states samples exactly like the oracle with
    those states."""
    import torch
    from paper_2509_11454_amd import percis as P
    g = W.rmat_graph(12, 8, seed=5, directed=False)
    rng = np.random.default_rng(7)
    c = P.Context(0)
    c.load_csr(g.n, g.row_ptr, g.col)
    og = O.Graph(g.n, g.row_ptr, g.col)
    for step in range(4):
        k = [W.uniform_states, W.skewed_states, W.beta_states, W.uniform_states][step](g.n, rng)
        if step == 2:
            c.set_states(torch.from_numpy(k.view(np.int16)).cuda())
        else:
            c.set_states(k)
        st = O.States(k)
        ho, so = oracle_hits(og, st, 0, 3000, 20 + step)
        hg, sg = gpu_hits(c, 0, 3000, 20 + step)
        assert np.array_equal(ho, hg), step
        same_stats(so, sg)
        if step == 1:
            with pytest.raises(P.PercisError) as e:
                c.set_states(np.full(g.n, 9, np.uint16))
            assert e.value.status == P.E_DEGENERATE
            with pytest.raises(P.PercisError) as e:
                c.sample(10, 1)
            assert e.value.status == P.E_STATE
    c.close()


def diameter_cases():
    rng = np.random.default_rng(3)
    out = [W.path_graph(300), W.star_graph(50), W.cycle_graph(101), W.grid_graph(40, 50), W.diamond_chain(30),
           W.complete_graph(20), W.complete_bipartite(5, 70)]
    out.append(disjoint_union([W.path_graph(30), W.grid_graph(7, 9), W.star_graph(200), W.cycle_graph(64)]))
    out.append(disjoint_union([W.er_graph(200, 210, 4), W.er_graph(3000, 3100, 5)]))   # many small components
    out.append(W.with_isolated_component(W.er_graph(300, 700, 9), 50)[0])
    out.append(W.rmat_graph(16, 8, seed=2, directed=False))
    out.append(W.rmat_graph(14, 8, seed=3, directed=True))
    out.append(W.random_small_graph(200, 0.01, 19, directed=True))
    out.append(disjoint_union([W.random_small_graph(60, 0.03, 20 + i, directed=True) for i in range(5)],
                              directed=True))
    out.append(W.prop7_instance(40)[0])
    out.append(W.csr_from_edges(6, np.zeros(0, np.int32), np.zeros(0, np.int32), False, name="no arcs"))
    # hub rows past the 1024-entry segments of the BFS (several segments, a ragged last one)
    out.append(W.star_graph(5000))
    out.append(disjoint_union([W.star_graph(3000), W.path_graph(40), W.star_graph(1025), W.star_graph(1024)]))
    del rng
    return out


@pytest.mark.parametrize("ci", range(18))
def test_vertex_diameter_matches_oracle(ci):
    """VertexDiamUB on the device equals the oracle's serial BFS/components
    bound (pinned on the CPU to the definition); an override replaces it and
    D < 0 restores it."""
    from paper_2509_11454_amd import percis as P
    g = diameter_cases()[ci]
    og = O.Graph(g.n, g.row_ptr, g.col, g.directed)
    want = O.vertex_diam_ub(og)
    c = P.Context(0)
    c.load_csr(g.n, g.row_ptr, g.col, directed=g.directed)
    assert c.vertex_diameter() == want, g.name
    c.set_vertex_diameter(want + 5)
    assert c.vertex_diameter() == want + 5
    c.set_vertex_diameter(-1)
    assert c.vertex_diameter() == want
    c.close()


def test_estimate_outputs_are_device_formula():
    """Algorithm 1's output p[v] = d_v h_v / l equals the device-built d_v
    times the phase-2 hits over l in IEEE double, bit for bit, and the
    phase-1 v_hat matches the oracle's loop over nodes to 1e-12."""
    g, k = W.workload_er1000()
    og, st = oracle_objects(g, k)
    c = gpu_context(g, k)
    eps, delta, seed = 0.02, 0.1, 9
    p, info = c.estimate(eps, delta, seed)
    d = c.debug_states()
    h2, _ = gpu_hits(c, 0, info["l"], seed, phase=2)
    want = d["d_v"] * h2.astype(np.float64) / float(info["l"])
    assert np.array_equal(p, want)
    rc, _, io = O.estimate(og, st, eps, delta, seed)
    assert rc == 0 and io["D"] == info["D"] and io["d_hat"] == info["d_hat"]
    assert abs(info["v_hat"] - io["v_hat"]) <= 1e-12 * io["v_hat"]
    c.close()
