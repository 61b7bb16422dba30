"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test states which definition it pins.  None of them re-derives an
expected value by calling the oracle routine it checks: the expected values
are hand-derived fixtures (tests/golden, each with its derivation), closed
forms, brute force over tiny inputs, or invariants computed independently
with numpy.
"""
import itertools

import numpy as np
import pytest

import gen
from conftest import golden, graph_from_fixture, ip_fixture_graph


# ----------------------------------------------------------------------------
# independent helpers (numpy, written for the tests)
# ----------------------------------------------------------------------------

def digit_distance_matrix(a, d):
    """D as a k x k matrix built top-down from mixed-radix digits (a_1 least
    significant): two PEs are at distance d_j where j is the highest level at
    which their digits differ."""
    a = list(a)
    k = int(np.prod(a))
    ids = np.arange(k)
    digits = []
    p = 1
    for ai in a:
        digits.append((ids // p) % ai)
        p *= ai
    D = np.zeros((k, k), dtype=np.int64)
    for j in range(len(a) - 1, -1, -1):
        differ = digits[j][:, None] != digits[j][None, :]
        D = np.where((D == 0) & differ, d[j], D)
    return D


def undirected_edges(g):
    src = np.repeat(np.arange(g.n), np.diff(g.xadj))
    keep = src < g.adjncy
    return src[keep], g.adjncy[keep].astype(np.int64), g.adjwgt[keep].astype(np.int64)


def j_undirected(g, part, D):
    u, v, w = undirected_edges(g)
    return int((w * D[part[u], part[v]]).sum())


def conn_table(g, part, k):
    """conn[v, x] = sum of edge weights from v to block x (dense, small k)."""
    src = np.repeat(np.arange(g.n), np.diff(g.xadj))
    c = np.zeros((g.n, k), dtype=np.int64)
    np.add.at(c, (src, part[g.adjncy]), g.adjwgt.astype(np.int64))
    return c


def small_random_graph(n, p, seed, wmax=5, cmax=1):
    rng = np.random.Generator(np.random.PCG64(seed))
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    if not pairs:
        pairs = [(0, 1)]
    e = np.array(pairs)
    w = rng.integers(1, wmax + 1, size=len(pairs))
    c = rng.integers(1, cmax + 1, size=n)
    return gen.from_edges(n, e[:, 0], e[:, 1], w, c)


HIERARCHIES = [((2, 2, 4), (1, 10, 100)), ((4, 8, 3), (1, 10, 100)),
               ((3, 5), (2, 7)), ((4,), (1,)), ((2, 3, 1, 2), (1, 4, 9, 20))]


# ----------------------------------------------------------------------------
# splitmix64 counter-based hash
# ----------------------------------------------------------------------------

def test_hash_is_published_splitmix64_stream(pmo):
    fx = golden("splitmix64.json")
    s0 = fx["streams"][0]
    assert [pmo.hash64(s0["seed"], i) for i in range(3)] == [int(h, 16) for h in s0["outputs_hex"]]
    s1 = fx["streams"][1]
    assert [pmo.hash64(s1["seed"], i) for i in range(5)] == s1["outputs"]


# ----------------------------------------------------------------------------
# D (Section 2, hierarchy and distances)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("a,d", HIERARCHIES)
def test_distance_matches_digit_matrix(pmo, a, d):
    D = digit_distance_matrix(a, d)
    k = D.shape[0]
    got = np.array([[pmo.distance(a, d, x, y) for y in range(k)] for x in range(k)])
    assert np.array_equal(got, D)


@pytest.mark.parametrize("a,d", [h for h in HIERARCHIES if list(h[1]) == sorted(h[1])])
def test_distance_is_ultrametric(pmo, a, d):
    k = pmo.num_pes(a)
    D = np.array([[pmo.distance(a, d, x, y) for y in range(k)] for x in range(k)])
    assert (np.diag(D) == 0).all()
    assert np.array_equal(D, D.T)
    # D(x,z) <= max(D(x,y), D(y,z)) for non-decreasing distances
    assert (D[:, None, :] <= np.maximum(D[:, :, None], D[None, :, :])).all()


def test_distance_row_sums_closed_form(pmo):
    for case in golden("distance_row_sums.json")["cases"]:
        a, d = case["a"], case["d"]
        k = pmo.num_pes(a)
        for x in {0, k // 2, k - 1}:
            assert sum(pmo.distance(a, d, x, y) for y in range(k)) == case["row_sum"]


# ----------------------------------------------------------------------------
# J (Section 2, GPMP objective)
# ----------------------------------------------------------------------------

def test_comm_cost_grid_tiling_closed_form(pmo):
    fx = golden("grid64_tiling.json")
    g = gen.grid2d(64, 64)
    i, j = np.arange(4096) // 64, np.arange(4096) % 64
    r, c = i // 16, j // 16
    pe = ((c & 1) + 2 * (r & 1) + 4 * (c >> 1) + 8 * (r >> 1)).astype(np.int32)
    assert np.bincount(pe).tolist() == [fx["block_size"]] * 16
    assert pmo.comm_cost(g, pe, (2, 2, 4), (1, 10, 100)) == fx["J_ordered"]
    u, v, _ = undirected_edges(g)
    assert int((pe[u] != pe[v]).sum()) == fx["cut_edges"]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_comm_cost_is_twice_undirected_sum(pmo, seed):
    a, d = (4, 8, 3), (1, 10, 100)
    g = gen.get("rgg14").graph()
    part = gen.random_mapping(g.n, 96, seed)
    J = pmo.comm_cost(g, part, a, d)
    assert J % 2 == 0
    assert J == 2 * j_undirected(g, part, digit_distance_matrix(a, d))


def test_unit_distances_reduce_to_edge_cut(pmo):
    g = gen.get("rmat14").graph()
    part = gen.random_mapping(g.n, 16, 5)
    u, v, w = undirected_edges(g)
    cut = int(w[part[u] != part[v]].sum())
    assert pmo.comm_cost(g, part, (2, 2, 4), (1, 1, 1)) == 2 * cut


# ----------------------------------------------------------------------------
# gains (equation (1))
# ----------------------------------------------------------------------------

def test_single_move_changes_J_by_twice_the_gain(pmo):
    a, d = (2, 2, 4), (1, 10, 100)
    g = gen.get("rmat14").graph()
    part = gen.random_mapping(g.n, 16, 9)
    rng = np.random.Generator(np.random.PCG64(3))
    J0 = pmo.comm_cost(g, part, a, d)
    for v in rng.integers(0, g.n, size=40):
        b = int(rng.integers(0, 16))
        moved = part.copy()
        moved[v] = b
        assert pmo.comm_cost(g, moved, a, d) == J0 - 2 * pmo.gain(g, part, a, d, int(v), b)


def test_gain_with_one_level_is_connectivity_difference(pmo):
    g = gen.get("rgg14").graph()
    part = gen.random_mapping(g.n, 8, 4)
    C = conn_table(g, part, 8)
    for v in range(0, g.n, 997):
        for b in range(8):
            expect = 3 * (C[v, b] - C[v, part[v]])
            assert pmo.gain(g, part, (8,), (3,), v, b) == expect


def level_projection_cost(C_row, b, a, d):
    """sum_x conn(v,x) D(b,x) via group sums S_i(b) over the level-i group of b
    (S_0 = conn(v,b), S_l = total): cost = sum_i d_i (S_i - S_{i-1})."""
    k = C_row.shape[0]
    S_prev = C_row[b]
    cost = 0
    p = 1
    for ai, di in zip(a, d):
        p *= ai
        grp = (np.arange(k) // p) == (b // p)
        S = C_row[grp].sum()
        cost += di * (S - S_prev)
        S_prev = S
    return cost


def test_gain_three_formulas_agree(pmo):
    a, d = (4, 8, 3), (1, 10, 100)
    k = 96
    g = gen.get("rmat14").graph()
    part = gen.random_mapping(g.n, k, 11)
    C = conn_table(g, part, k)
    # formula 2: the first-filter gains produced by a label-propagation round
    _, _, target, gain, _ = pmo.lp_round(g, a, d, part, np.zeros(g.n, np.uint8))
    checked = 0
    for v in range(0, g.n, 61):
        blocks = np.nonzero(C[v])[0]
        cand = [b for b in blocks if b != part[v]]
        if not cand:
            assert gain[v] == np.iinfo(np.int64).min
            continue
        own = level_projection_cost(C[v], part[v], a, d)
        g3 = {b: own - level_projection_cost(C[v], b, a, d) for b in cand}
        for b in cand:
            assert pmo.gain(g, part, a, d, v, int(b)) == g3[b]          # formula 1
        best = max(cand, key=lambda b: (g3[b], -b))
        if g3[best] >= 0:
            assert (target[v], gain[v]) == (best, g3[best])
            checked += 1
        else:
            assert gain[v] == np.iinfo(np.int64).min
    assert checked > 10


# ----------------------------------------------------------------------------
# label propagation (Algorithm 4)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("fixture", ["lp_round_p7.json", "lp_round_earlier_member.json"])
def test_lp_round_hand_examples(pmo, fixture):
    fx = golden(fixture)
    g = graph_from_fixture(fx)
    a, d = fx["a"], fx["d"]
    part0 = np.array(fx["part_in"], np.int32)
    assert pmo.comm_cost(g, part0, a, d) == fx["J_before"]
    part, lock, target, gain, moved = pmo.lp_round(g, a, d, part0, np.zeros(g.n, np.uint8))
    nin = np.iinfo(np.int64).min
    assert [None if x == nin else int(x) for x in gain] == fx["gain"]
    assert target.tolist() == fx["target"]
    assert moved.tolist() == fx["moved"]
    assert lock.tolist() == fx["moved"]
    assert part.tolist() == fx["part_out"]
    assert pmo.comm_cost(g, part, a, d) == fx["J_after"]


def test_lp_locked_vertices_do_not_move(pmo):
    fx = golden("lp_round_p7.json")
    g = graph_from_fixture(fx)
    lock = np.array([1, 0, 0, 0], np.uint8)
    part, lock2, target, gain, moved = pmo.lp_round(g, fx["a"], fx["d"], fx["part_in"], lock)
    # 0 is locked, so 1 is alone in X: it re-evaluates to 40 and moves to block 0
    assert gain[0] == np.iinfo(np.int64).min and gain[1] == 40
    assert moved.tolist() == [0, 1, 0, 0]
    assert part.tolist() == [0, 0, 0, 2]


def test_lp_round_sequential_replay_telescopes(pmo):
    """Applying the moved set one vertex at a time in the implicit order, each
    move's exact gain in the state before it adds up to the J difference."""
    a, d = (4, 8, 8), (1, 10, 100)
    g = gen.get("rgg14").graph()
    part0 = gen.random_balanced_mapping(g.n, 256, 7)
    part, _, target, gain, moved = pmo.lp_round(g, a, d, part0, np.zeros(g.n, np.uint8))
    order = sorted(np.nonzero(moved)[0], key=lambda v: (-gain[v], v))
    state = part0.copy()
    total = 0
    for v in order:
        total += pmo.gain(g, state, a, d, int(v), int(target[v]))
        state[v] = target[v]
    assert np.array_equal(state, part)
    assert pmo.comm_cost(g, part0, a, d) - pmo.comm_cost(g, part, a, d) == 2 * total


# ----------------------------------------------------------------------------
# rebalancing (Algorithm 5 and the text around it)
# ----------------------------------------------------------------------------

def test_weak_rebalance_hand_example(pmo):
    fx = golden("weak_rebalance_buckets.json")
    g = graph_from_fixture(fx)
    total, k = int(g.vwgt.sum()), 2
    lm = pmo.lmax(total, k, fx["eps"])
    sg = pmo.sigma(lm, total, k)
    assert (lm, sg) == (3, 3)
    for seed in (1, 2, 3):
        part, moved = pmo.rebalance(g, k, fx["part_in"], False, lm, sg, seed, 0, 1)
        assert moved.tolist() == fx["moved"]
        assert part.tolist() == fx["part_out"]


def test_strong_rebalance_balances_unit_weights(pmo):
    g = gen.get("rgg14").graph()
    k, a, d = 64, (4, 4, 4), (1, 10, 100)
    total = int(g.vwgt.sum())
    lm = pmo.lmax(total, k, 0.03)
    sg = pmo.sigma(lm, total, k)
    part = gen.random_mapping(g.n, k, 3)
    part[: g.n // 8] = 0  # overload block 0 heavily
    w0 = pmo.block_weights(g, part, k)
    assert w0.max() > lm
    p2, moved = pmo.rebalance(g, k, part, True, lm, sg, 1, 0, 1)
    w1 = pmo.block_weights(g, p2, k)
    assert w1.max() <= lm


def test_strong_rebalance_weighted_hand_example(pmo):
    fx = golden("strong_rebalance_weighted.json")
    g = graph_from_fixture(fx)
    k = int(np.prod(fx["a"]))
    total = int(g.vwgt.sum())
    lm = pmo.lmax(total, k, fx["eps"])
    assert lm == fx["lmax"]
    sg = pmo.sigma(lm, total, k)
    for seed in (1, 2, 3):
        part, moved = pmo.rebalance(g, k, fx["part_in"], True, lm, sg, seed, 0, 3)
        assert moved.tolist() == fx["moved"]
        assert part.tolist() == fx["part_out"]
        assert pmo.block_weights(g, part, k).tolist() == fx["weights_out"]


@pytest.mark.parametrize("name,k", [("rmat14", 512), ("rmat14", 64), ("rmat17", 512)])
def test_strong_rebalance_never_overloads_and_balances(pmo, name, k):
    """Strong rebalancing must not overload a destination and balances in
    one round (Section 4.2, 'Rebalancing'), here on graphs with vertex
    weights 1..4 from a start with one block holding 5 % of all vertices
    besides its random share."""
    g = gen.get(name).graph()
    total = int(g.vwgt.sum())
    lm = pmo.lmax(total, k, 0.03)
    sg = pmo.sigma(lm, total, k)
    rng = np.random.default_rng(5)
    part = rng.integers(0, k, g.n).astype(np.int32)
    part[rng.random(g.n) < 0.05] = 3
    w0 = pmo.block_weights(g, part, k)
    assert w0.max() > lm
    p2, moved = pmo.rebalance(g, k, part, True, lm, sg, 7, 0, 1)
    w1 = pmo.block_weights(g, p2, k)
    # no block at or below L_max before the round is above it afterwards
    assert not np.any((w0 <= lm) & (w1 > lm))
    # the blocks' free capacity covers the excess here: one round balances
    assert w1.max() <= lm
    assert np.array_equal(moved != 0, p2 != part)


def test_heavy_vertex_boundary_hand_example(pmo):
    fx = golden("heavy_vertex_boundary.json")
    g = graph_from_fixture(fx)
    k = int(np.prod(fx["a"]))
    total = int(g.vwgt.sum())
    lm = pmo.lmax(total, k, fx["eps"])
    sg = pmo.sigma(lm, total, k)
    assert (lm, sg) == (1030, 1000)
    part, moved = pmo.rebalance(g, k, fx["part_in"], False, lm, sg, 1, 0, 1)
    assert moved.tolist() == fx["weak_moved"] and part.tolist() == fx["weak_part_out"]
    part, moved = pmo.rebalance(g, k, fx["part_in"], True, lm, sg, 1, 0, 1)
    assert moved.tolist() == fx["strong_moved"] and part.tolist() == fx["strong_part_out"]


@pytest.mark.parametrize("case", [0, 1])
def test_refine_patience_and_phi_hand_example(pmo, case):
    fx = golden("refine_patience.json")
    c = fx["cases"][case]
    g = graph_from_fixture({"n": fx["n"], "vwgt": fx["vwgt"], "edges": c["edges"]})
    rc, part, st, kinds, ja, ia, ct = pmo.refine_trace(g, fx["a"], fx["d"], fx["eps"], 1,
                                                       fx["part_in"])
    assert rc == 0
    assert kinds == c["kinds"]
    assert ct.tolist() == c["counter"]
    assert ja.tolist() == c["j_after"]
    assert part.tolist() == c["part_out"]


def test_refine_weak_strong_order_hand_example(pmo):
    fx = golden("refine_weak_strong_order.json")
    g = graph_from_fixture(fx)
    rc, part, st, kinds, ja, ia, ct = pmo.refine_trace(g, fx["a"], fx["d"], fx["eps"], 1,
                                                       fx["part_in"])
    assert rc == fx["status"]
    assert kinds == fx["kinds"]
    assert ct.tolist() == fx["counter"]
    assert ia.tolist() == fx["imb_after"]
    assert part.tolist() == fx["part_out"] and st.maxw_final == fx["maxw_final"]


def test_weak_rebalance_moves_only_from_overloaded(pmo):
    g = gen.get("rmat14").graph()
    k = 128
    total = int(g.vwgt.sum())
    lm = pmo.lmax(total, k, 0.03)
    sg = pmo.sigma(lm, total, k)
    part = gen.random_mapping(g.n, k, 8)
    w0 = pmo.block_weights(g, part, k)
    p2, moved = pmo.rebalance(g, k, part, False, lm, sg, 1, 0, 1)
    mv = moved.astype(bool)
    assert (w0[part[mv]] > lm).all()
    assert (w0[p2[mv]] <= sg).all()
    # moved weight per source block covers the excess by less than one vertex
    w1 = pmo.block_weights(g, p2, k)
    out = np.bincount(part[mv], weights=g.vwgt[mv], minlength=k).astype(np.int64)
    over = w0 > lm
    # the moved prefix stops as soon as it covers the excess
    assert (out[over] < (w0 - lm)[over] + g.vwgt.max()).all()
    assert (out[over] > 0).all()
    assert w1.sum() == w0.sum()


# ----------------------------------------------------------------------------
# refinement controller (Algorithm 6)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("name,seed", [("grid64", 1), ("rgg14", 2), ("rmat14", 3)])
def test_refine_balance_invariant_and_monotone(pmo, name, seed):
    w = gen.get(name)
    g = w.graph()
    total = int(g.vwgt.sum())
    lm = pmo.lmax(total, w.k, w.eps)
    start = gen.random_balanced_mapping(g.n, w.k, seed)
    if pmo.block_weights(g, start, w.k).max() > lm:
        start = pmo.initial_partition(g, w.a)
    rc, part, st = pmo.refine(g, w.a, w.d, w.eps, seed, start)
    wb = pmo.block_weights(g, part, w.k)
    J = pmo.comm_cost(g, part, w.a, w.d)
    assert st.j_final == J and st.maxw_final == wb.max()
    if pmo.block_weights(g, start, w.k).max() <= lm:
        assert rc == 0 and wb.max() <= lm
        assert J <= st.j_initial
    assert np.bincount(part, minlength=w.k).sum() == g.n


def test_refine_from_imbalanced_start_reaches_balance(pmo):
    w = gen.get("rgg14")
    g = w.graph()
    start = gen.random_mapping(g.n, w.k, 1)
    start[: g.n // 4] = 3
    rc, part, st = pmo.refine(g, w.a, w.d, w.eps, 5, start)
    lm = pmo.lmax(int(g.vwgt.sum()), w.k, w.eps)
    assert rc == 0 and pmo.block_weights(g, part, w.k).max() <= lm
    assert st.weak_iterations + st.strong_iterations > 0


def brute_force(g, a, d, eps, pmo):
    D = digit_distance_matrix(a, d)
    k = D.shape[0]
    n = g.n
    lm = pmo.lmax(int(g.vwgt.sum()), k, eps)
    u, v, w = undirected_edges(g)
    all_maps = np.array(list(itertools.product(range(k), repeat=n)), dtype=np.int64)
    J = 2 * (w[None, :] * D[all_maps[:, u], all_maps[:, v]]).sum(axis=1)
    wts = np.zeros((all_maps.shape[0], k), np.int64)
    for b in range(k):
        wts[:, b] = ((all_maps == b) * g.vwgt[None, :]).sum(axis=1)
    ok = wts.max(axis=1) <= lm
    best = np.argmin(np.where(ok, J, np.iinfo(np.int64).max))
    return int(J[best]), all_maps[best].astype(np.int32)


@pytest.mark.parametrize("n,seed", [(6, 1), (7, 2), (8, 3), (8, 4)])
def test_brute_force_optimum(pmo, n, seed):
    a, d, eps = (2, 2), (1, 10), 0.03
    g = small_random_graph(n, 0.5, seed, wmax=6)
    Jstar, pstar = brute_force(g, a, d, eps, pmo)
    rc, part, st = pmo.map_graph(g, a, d, eps, seed)
    assert rc == 0
    assert pmo.comm_cost(g, part, a, d) >= Jstar
    # refining an optimal mapping returns it unchanged, after exactly 12 loop
    # bodies: no feasible mapping is cheaper and no unbalanced one is
    # lighter than a balanced best, so the counter never restarts
    rc2, part2, st2 = pmo.refine(g, a, d, eps, seed, pstar)
    assert rc2 == 0 and np.array_equal(part2, pstar) and st2.j_final == Jstar
    assert st2.iterations == 12


# ----------------------------------------------------------------------------
# order invariance (rows shuffled -> identical results)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["grid64", "rgg14", "rmat14"])
def test_row_order_invariance(pmo, name):
    w = gen.get(name)
    g = w.graph()
    gs = gen.shuffle_rows(g, 99)
    rc1, p1, s1 = pmo.map_graph(g, w.a, w.d, w.eps, 3)
    rc2, p2, s2 = pmo.map_graph(gs, w.a, w.d, w.eps, 3)
    assert rc1 == rc2 and np.array_equal(p1, p2) and s1.j_final == s2.j_final


# ----------------------------------------------------------------------------
# matching and contraction (Section 4.2)
# ----------------------------------------------------------------------------

def test_two_hop_matching_properties(pmo):
    fx = golden("two_hop_matching.json")
    g = graph_from_fixture(fx)
    for seed in range(1, 9):
        _, m = pmo.hem(g, fx["lmax"], seed)
        assert np.array_equal(m[m], np.arange(g.n))
        nb = [set(g.adjncy[g.xadj[x]:g.xadj[x + 1]].tolist()) for x in range(g.n)]
        for x in range(g.n):
            y = int(m[x])
            if y == x or y in nb[x]:
                continue
            assert (nb[x] & nb[y]) or (not nb[x] and not nb[y])
        # 9 is the only isolated vertex: no twin partner
        assert m[9] == 9
        # leaves 3 and 4 (neighbour 0) pair up whenever both are still unmatched leaves
        if m[3] != 0 and m[4] != 0:
            assert m[3] == 4


def test_two_hop_leaf_twin_relative_closed_cases(pmo):
    """Hand cases where heavy-edge matching cannot act and each two-hop
    category decides alone."""
    # leaves: star with 4 leaves, centre heavier than L_max allows to pair
    g = gen.from_edges(5, [0, 0, 0, 0], [1, 2, 3, 4], [1, 1, 1, 1], [9, 1, 1, 1, 1])
    _, m = pmo.hem(g, 5, 1)
    assert m.tolist() == [0, 2, 1, 4, 3]
    # twins: K_{2,3} -- 2,3,4 all see {0,1}; the heavy vertices 0,1 (weight 9)
    # fit no pair under L_max 9; relatives then group 0 and 1 (matchmaker 2)
    # but their pair is too heavy
    g = gen.from_edges(5, [0, 0, 0, 1, 1, 1], [2, 3, 4, 2, 3, 4], [1] * 6, [9, 9, 1, 1, 1])
    _, m = pmo.hem(g, 9, 1)
    assert m.tolist() == [0, 1, 3, 2, 4]
    # relatives: path 0-1-2 with centre too heavy: 0 and 2 share neighbour 1
    # but are leaves (degree 1) -> paired already as leaves of 1
    g = gen.from_edges(4, [0, 1, 1], [1, 2, 3], [1, 1, 1], [1, 9, 1, 1])
    _, m = pmo.hem(g, 5, 1)
    assert m.tolist() == [2, 1, 0, 3]
    # relatives proper: light 0 (neighbours 1,4) and 3 (neighbours 1,5) are
    # not twins; their smallest-degree neighbour is 1 (degree 2 < 3), so they
    # form one relative group; heavy 1,2,4,5 (weight 9) fit no pair
    g = gen.from_edges(6, [0, 0, 3, 3, 4, 4, 5], [1, 4, 1, 5, 5, 2, 2], [1] * 7,
                       [1, 9, 9, 1, 9, 9])
    _, m = pmo.hem(g, 5, 1)
    assert m.tolist() == [3, 1, 2, 0, 4, 5]


def test_hem_hand_example(pmo):
    fx = golden("hem_rating.json")
    g = graph_from_fixture(fx)
    rounds, match = pmo.hem(g, fx["lmax"], 1)
    assert match.tolist() == fx["match"] and rounds == fx["rounds"]


@pytest.mark.parametrize("name", ["grid64", "rgg14", "rmat14"])
def test_hem_matching_properties(pmo, name):
    w = gen.get(name)
    g = w.graph()
    lm = pmo.lmax(int(g.vwgt.sum()), w.k, w.eps)
    rounds, match = pmo.hem(g, lm, 7)
    assert rounds < 64
    v = np.arange(g.n)
    assert np.array_equal(match[match], v)                      # an involution
    paired = match != v
    assert (g.vwgt[v[paired]] + g.vwgt[match[paired]] <= lm).all()
    deg = np.diff(g.xadj)
    # pairs are edges, or two-hop pairs (a common neighbour), or isolated twins
    src = np.repeat(v, deg)
    is_edge = set(zip(src.tolist(), g.adjncy.tolist()))
    nbrs = [set(g.adjncy[g.xadj[x]:g.xadj[x + 1]].tolist()) for x in range(g.n)]
    for x in v[paired]:
        y = int(match[x])
        if (int(x), y) in is_edge:
            continue
        if deg[x] == 0:
            assert deg[y] == 0
        else:
            assert nbrs[int(x)] & nbrs[y], (x, y)
    # maximality: no eligible edge joins two unmatched vertices
    un = ~paired
    both = un[src] & un[g.adjncy] & (g.vwgt[src] + g.vwgt[g.adjncy] <= lm)
    assert not both.any()


@pytest.mark.parametrize("name", ["grid64", "rgg14", "rmat14"])
def test_contraction_properties(pmo, name):
    w = gen.get(name)
    g = w.graph()
    lm = pmo.lmax(int(g.vwgt.sum()), w.k, w.eps)
    _, match = pmo.hem(g, lm, 7)
    nc, cmap = pmo.coarse_map(match)
    # coarse ids: ranks of the smaller member, so cmap is non-decreasing over leaders
    leaders = np.nonzero(match >= np.arange(g.n))[0]
    assert np.array_equal(cmap[leaders], np.arange(nc))
    assert np.array_equal(cmap, cmap[match])
    cx, ca, cw, cv = pmo.contract(g, cmap, nc)
    cg = gen.Graph(cx, ca, cw, cv)
    assert cv.sum() == g.vwgt.sum()
    # arc weight: every matched edge (both arcs) disappears, nothing else
    v = np.arange(g.n)
    src = np.repeat(v, np.diff(g.xadj))
    internal = g.adjwgt[(match[src] == g.adjncy)].sum()
    assert cw.astype(np.int64).sum() == g.adjwgt.astype(np.int64).sum() - internal
    # symmetric rows, no self-loops, no duplicates
    csrc = np.repeat(np.arange(nc), np.diff(cx))
    assert (csrc != ca).all()
    fw = dict(zip(zip(csrc.tolist(), ca.tolist()), cw.tolist()))
    assert len(fw) == len(ca)
    assert all(fw[(y, x)] == wt for (x, y), wt in fw.items())
    # the objective and block weights survive projection
    for seed in (1, 2):
        pc = gen.random_mapping(nc, w.k, seed)
        pf = pc[cmap]
        assert pmo.comm_cost(cg, pc, w.a, w.d) == pmo.comm_cost(g, pf, w.a, w.d)
        assert np.array_equal(pmo.block_weights(cg, pc, w.k), pmo.block_weights(g, pf, w.k))


def _contract_by_definition(g, cmap, nc):
    """Coarse graph written out from its definition: per coarse row, the sum
    of the weights of the fine arcs to every other coarse vertex, rows
    ascending by neighbour, vertex weights summed."""
    rows = [dict() for _ in range(nc)]
    for v in range(g.n):
        c = int(cmap[v])
        for e in range(int(g.xadj[v]), int(g.xadj[v + 1])):
            cu = int(cmap[int(g.adjncy[e])])
            if cu != c:
                rows[c][cu] = rows[c].get(cu, 0) + int(g.adjwgt[e])
    cx = np.zeros(nc + 1, np.int64)
    ca, cw = [], []
    for c in range(nc):
        for cu in sorted(rows[c]):
            ca.append(cu)
            cw.append(rows[c][cu])
        cx[c + 1] = len(ca)
    cv = np.zeros(nc, np.int64)
    np.add.at(cv, cmap, g.vwgt.astype(np.int64))
    return cx, np.array(ca, np.int64), np.array(cw, np.int64), cv


def _twin_hubs(leaves, seed):
    rng = np.random.default_rng(seed)
    lv = 2 + np.arange(leaves)
    u = np.concatenate([[0], np.zeros(leaves, np.int64), np.ones(leaves, np.int64)])
    v = np.concatenate([[1], lv, lv])
    g = gen.from_edges(leaves + 2, u, v, rng.integers(1, 11, u.shape[0]),
                       rng.integers(1, 5, leaves + 2))
    m = np.arange(leaves + 2, dtype=np.int32)
    m[[0, 1]] = [1, 0]
    return g, m


def _pairs_only(n, seed):
    rng = np.random.default_rng(seed)
    u = np.arange(0, n, 2)
    g = gen.from_edges(n, u, u + 1, rng.integers(1, 11, n // 2), np.ones(n))
    return g, np.arange(n, dtype=np.int32) ^ 1


@pytest.mark.parametrize("case", ["hem_rgg14", "identity_rmat14", "twin_hubs", "pairs_only"])
def test_contraction_equals_definition(pmo, case):
    """The oracle's contraction against the coarse graph written out from its
    definition (brute force), on matchings of the matcher, no matching, two
    matched hubs sharing every neighbour (each merged arc adds two weights)
    and a matching that leaves no coarse arc."""
    if case == "hem_rgg14":
        w = gen.get("rgg14")
        g = w.graph()
        _, match = pmo.hem(g, pmo.lmax(int(g.vwgt.sum()), w.k, w.eps), 3)
    elif case == "identity_rmat14":
        g = gen.get("rmat14").graph()
        match = np.arange(g.n, dtype=np.int32)
    elif case == "twin_hubs":
        g, match = _twin_hubs(300, 4)
    else:
        g, match = _pairs_only(600, 5)
    nc, cmap = pmo.coarse_map(match)
    got = pmo.contract(g, cmap, nc)
    exp = _contract_by_definition(g, cmap, nc)
    for x, y in zip(got, exp):
        assert np.array_equal(np.asarray(x, np.int64), y)
    if case == "twin_hubs":
        assert exp[0][1] - exp[0][0] == 300          # the hub pair's row: every leaf once
    if case == "pairs_only":
        assert exp[0][-1] == 0 and nc == 300


# ----------------------------------------------------------------------------
# initial partitioning and the multilevel driver
# ----------------------------------------------------------------------------

def test_initial_partition_path_closed_form(pmo):
    fx = golden("ip_path16.json")
    g = gen.path_graph(fx["n"])
    part = pmo.initial_partition(g, fx["a"])
    assert part.tolist() == fx["part"]
    assert pmo.comm_cost(g, part, fx["a"], fx["d"]) == fx["J_ordered"]


@pytest.mark.parametrize("fixture", ["ip_star16.json", "ip_two_paths16.json"])
def test_initial_partition_restart_closed_forms(pmo, fixture):
    # the breadth-first order visits neighbours in ascending order and
    # restarts at the smallest unvisited id (a half without inner edges, a
    # second component); every cut is at the exact proportional weight
    fx = golden(fixture)
    g = ip_fixture_graph(fx)
    part = pmo.initial_partition(g, fx["a"])
    assert part.tolist() == fx["part"]
    assert pmo.comm_cost(g, part, fx["a"], fx["d"]) == fx["J_ordered"]


def test_initial_partition_balance(pmo):
    g = gen.get("rgg14").graph()
    a = (4, 8, 8)
    part = pmo.initial_partition(g, a)
    w = np.bincount(part, minlength=256)
    # every split cuts at the exact proportional weight: within one vertex per level
    assert w.max() - w.min() <= 2 * len(a)


@pytest.mark.parametrize("name,seed", [("grid64", 1), ("grid64", 2), ("rgg14", 1), ("rmat14", 1)])
def test_map_balance_and_levels(pmo, name, seed):
    w = gen.get(name)
    g = w.graph()
    rc, part, st = pmo.map_graph(g, w.a, w.d, w.eps, seed)
    lm = pmo.lmax(int(g.vwgt.sum()), w.k, w.eps)
    assert st.lmax == lm
    assert rc == 0 and pmo.block_weights(g, part, w.k).max() <= lm
    assert st.j_final == pmo.comm_cost(g, part, w.a, w.d)
    ns = list(st.level_n[: st.levels])
    assert ns[0] == g.n and all(x > y for x, y in zip(ns, ns[1:]))
    for x, y in zip(ns, ns[1:]):
        assert 20 * y <= 19 * x
    # coarsening stops once fewer than 8k vertices remain (Section 4.2,
    # initial partitioning), and not before
    assert all(x >= 8 * w.k for x in ns[:-1])
    if len(ns) > 1:
        assert ns[-1] < 8 * w.k


# ----------------------------------------------------------------------------
# refinement variants (Section 4.2): Jet's relaxed first filter, J-objective
# rebalancing
# ----------------------------------------------------------------------------

def test_jet_filter_hand_example(pmo):
    # edges (0,1) w 3, (0,2) w 2; blocks [0,0,1,1]; l = 1, d = 1 (gain =
    # conn(b) - conn(own)).  Vertex 0: gain to block 1 is 2 - 3 = -1, so it
    # enters X only when -G = 1 < floor(c * conn(0, own) = c * 3): c = 1 yes,
    # c = 1/2 no.  Vertex 2: gain 2 - 0 = 2.  Phase 2: vertex 2 ranks before
    # vertex 0 (higher gain); 0's re-evaluated gain counts 2 at block 0:
    # 3*(0-1) + 2*(0-1) = -5 < 0; 2's counts 0 at its block 0: 2*(1-0) = 2.
    g = gen.from_edges(4, [0, 0], [1, 2], [3, 2], [1, 1, 1, 1])
    part0 = [0, 0, 1, 1]
    nin = np.iinfo(np.int64).min
    for c, gains, targets in (((1, 1), [-1, nin, 2, nin], [1, 0, 0, 1]),
                              ((1, 2), [nin, nin, 2, nin], [0, 0, 0, 1])):
        part, lock, target, gain, moved = pmo.lp_round(g, (2,), (1,), part0, [0] * 4,
                                                       pmo.variants(jet_c=c))
        assert gain.tolist() == gains, c
        assert target.tolist() == targets, c
        assert moved.tolist() == [0, 0, 1, 0]
        assert part.tolist() == [0, 0, 0, 1]


@pytest.mark.parametrize("name", ["rgg14", "rmat14"])
def test_jet_filter_with_vanishing_c_is_the_standard_method(pmo, name):
    # floor(c * conn) = 0 for every vertex, so no negative move passes
    w = gen.get(name)
    g = w.graph()
    base = pmo.map_graph(g, w.a, w.d, w.eps, 1)
    var = pmo.map_graph(g, w.a, w.d, w.eps, 1, pmo.variants(jet_c=(1, 1 << 30)))
    assert base[0] == var[0] and base[2].j_final == var[2].j_final
    assert np.array_equal(base[1], var[1])


@pytest.mark.parametrize("strong", [False, True])
def test_j_rebalance_with_one_unit_level_is_edge_cut_rebalance(pmo, strong):
    # l = 1, d = 1: G_b(v) = conn(v,b) - conn(v,Pi(v)), the edge-cut loss
    g = gen.get("rmat14").graph()
    k = 64
    total = int(g.vwgt.sum())
    lm = pmo.lmax(total, k, 0.03)
    sg = pmo.sigma(lm, total, k)
    part = gen.random_mapping(g.n, k, 5)
    part[: g.n // 10] = 3
    std = pmo.rebalance(g, k, part, strong, lm, sg, 7, 0, 1)
    var = pmo.rebalance(g, k, part, strong, lm, sg, 7, 0, 1, a=(k,), d=(1,),
                        var=pmo.variants(j_rebalance=True))
    assert np.array_equal(std[0], var[0]) and np.array_equal(std[1], var[1])
    base = pmo.map_graph(g, (k,), (1,), 0.03, 2)
    jv = pmo.map_graph(g, (k,), (1,), 0.03, 2, pmo.variants(j_rebalance=True))
    assert np.array_equal(base[1], jv[1]) and base[2].j_final == jv[2].j_final


def test_j_rebalance_destinations_maximise_the_gain(pmo):
    # every mover of a weak J-objective round goes to the eligible neighbour
    # block of largest gain (eq. 1, pmo_gain), smaller id on ties, or, without
    # one, to some block within sigma
    g = gen.get("rgg14").graph()
    a, d = (4, 4, 4), (1, 10, 100)
    k = 64
    total = int(g.vwgt.sum())
    lm = pmo.lmax(total, k, 0.03)
    sg = pmo.sigma(lm, total, k)
    part = gen.random_balanced_mapping(g.n, k, 4)
    # overload block 9 with vertices spread over the whole graph, so that its
    # sources have other neighbour blocks
    part[np.random.Generator(np.random.PCG64(6)).choice(g.n, g.n // 16, replace=False)] = 9
    w0 = pmo.block_weights(g, part, k)
    p2, moved = pmo.rebalance(g, k, part, False, lm, sg, 3, 0, 1, a=a, d=d,
                              var=pmo.variants(j_rebalance=True))
    mv = np.nonzero(moved)[0]
    assert len(mv) > 0
    checked = 0
    for v in mv[:400]:
        nb = {int(part[u]) for u in g.adjncy[g.xadj[v]:g.xadj[v + 1]]}
        cand = sorted(b for b in nb if b != part[v] and w0[b] <= sg)
        if cand:
            gains = [pmo.gain(g, part, a, d, int(v), b) for b in cand]
            best = cand[int(np.argmax(gains))]  # first maximum = smaller id
            assert p2[v] == best
            checked += 1
        else:
            assert w0[p2[v]] <= sg
    assert checked > 0


# ----------------------------------------------------------------------------
# hierarchical multisection (Section 4.1, Algorithms 1 and 2)
# ----------------------------------------------------------------------------

def test_subgraphs_hand_example(pmo):
    # path 0-1-2-3-4 (weights 1..4), blocks [1,0,1,1,0]: block 0 = {1,4} with
    # no inner edge; block 1 = {0,2,3} with the edge 2-3 (weight 3) only
    g = gen.from_edges(5, [0, 1, 2, 3], [1, 2, 3, 4], [1, 2, 3, 4], [5, 6, 7, 8, 9])
    s = pmo.subgraphs(g, [1, 0, 1, 1, 0], 2)
    assert s["vstart"].tolist() == [0, 2, 5]
    assert s["estart"].tolist() == [0, 0, 2]
    assert s["order"].tolist() == [1, 4, 0, 2, 3]
    # block 0 rows at xadj[0..2], block 1 rows at xadj[3..6]
    assert s["xadj"].tolist() == [0, 0, 0, 0, 0, 1, 2]
    assert s["adjncy"].tolist() == [2, 1]          # local ids: 2 -> 1, 3 -> 2
    assert s["adjwgt"].tolist() == [3, 3]
    assert s["vwgt"].tolist() == [6, 9, 5, 7, 8]


@pytest.mark.parametrize("name", ["rgg14", "rmat14"])
def test_subgraphs_are_the_induced_subgraphs(pmo, name):
    g = gen.get(name).graph()
    parts = 7
    part = gen.random_mapping(g.n, parts, 9)
    s = pmo.subgraphs(g, part, parts)
    src = np.repeat(np.arange(g.n), np.diff(g.xadj))
    inner = part[src] == part[g.adjncy]
    assert s["estart"][-1] == int(inner.sum())
    for b in range(parts):
        lo, hi = s["vstart"][b], s["vstart"][b + 1]
        verts = s["order"][lo:hi]
        assert np.array_equal(verts, np.nonzero(part == b)[0])   # id order
        x = s["xadj"][lo + b: hi + b + 1]
        adj = s["adjncy"][s["estart"][b]: s["estart"][b + 1]]
        wgt = s["adjwgt"][s["estart"][b]: s["estart"][b + 1]]
        for j in range(0, len(verts), max(1, len(verts) // 50)):
            v = verts[j]
            row = g.adjncy[g.xadj[v]:g.xadj[v + 1]]
            keep = part[row] == b
            assert np.array_equal(verts[adj[x[j]:x[j + 1]]], row[keep])
            assert np.array_equal(wgt[x[j]:x[j + 1]], g.adjwgt[g.xadj[v]:g.xadj[v + 1]][keep])


def test_adaptive_imbalance_closed_forms(pmo):
    # top level of l = 3 with eps = 3 %: 1.03^(1/3) - 1 = 0.00990163...
    assert pmo.adaptive_eps_ppm(30000, 256, 256, 1000, 1000, 3) == 9902
    # one level left, a subgraph of exactly its share: eps unchanged
    assert pmo.adaptive_eps_ppm(30000, 8, 256, 32000, 1000, 1) == 30000
    # a subgraph 1 % heavier than its share, two levels left
    want = round(((1.03 * 64 * 100000) / (256 * 25250)) ** 0.5 * 1e6 - 1e6)
    assert pmo.adaptive_eps_ppm(30000, 64, 256, 100000, 25250, 2) == want
    # never negative
    assert pmo.adaptive_eps_ppm(30000, 8, 256, 32000, 2000, 1) == 0


@pytest.mark.parametrize("name", ["grid64", "rgg14"])
def test_hm_with_one_level_is_the_edge_cut_partitioner(pmo, name):
    g = gen.get(name).graph()
    rc, part = pmo.hm(g, (16,), 0.03, 3)
    rc2, part2, _ = pmo.map_graph(g, (16,), (1,), 0.03, 3)
    assert rc == rc2 and np.array_equal(part, part2)


@pytest.mark.parametrize("name,a", [("rgg14", (4, 8, 8)), ("rmat14", (4, 16, 8)),
                                    ("grid64", (2, 2, 4)), ("rgg14", (4, 8, 3))])
def test_hm_is_hierarchical_and_balanced(pmo, name, a):
    g = gen.get(name).graph()
    k = int(np.prod(a))
    rc, part = pmo.hm(g, a, 0.03, 1)
    assert part.min() >= 0 and part.max() < k
    # the top-level digit is one partition of the whole graph into a_l blocks:
    # it equals the edge-cut partitioner with the adaptive imbalance of the
    # top level
    top = part // (k // a[-1])
    ppm = pmo.adaptive_eps_ppm(30000, k, k, int(g.vwgt.sum()), int(g.vwgt.sum()), len(a))
    rc2, top2, _ = pmo.map_graph(g, (a[-1],), (1,), ppm / 1e6, 1)
    assert np.array_equal(top, top2)
    if rc == 0:
        w = pmo.block_weights(g, part, k)
        assert w.max() <= pmo.lmax(int(g.vwgt.sum()), k, 0.03)


# ----------------------------------------------------------------------------
# the "ultra" repetition (Section 5: Jet's ultra configuration runs the complete
# refinement 18 times): Algorithm 6 runs `repeats` times per level
# ----------------------------------------------------------------------------

def test_ultra_one_run_is_the_method(pmo):
    w = gen.get("rgg14")
    g = w.graph()
    base = pmo.map_graph(g, w.a, w.d, w.eps, 3)
    for r in (0, 1):
        rc, part, st = pmo.map_graph(g, w.a, w.d, w.eps, 3, pmo.variants(repeats=r))
        assert rc == base[0] and np.array_equal(part, base[1]) and st.j_final == base[2].j_final


def test_ultra_single_level_is_refinement_repeated(pmo):
    """Below 8k vertices nothing is coarsened: the map is the initial
    partition refined; with repeats R it is that refinement run R times, run r
    from run r - 1's result with seed + r."""
    g = gen.grid2d(10, 11)
    a, d, eps = (2, 2, 4), (1, 10, 100), 0.03     # k = 16: 110 < 8k, one level
    part = pmo.initial_partition(g, a)
    for r in range(3):
        rc_r, part, st_r = pmo.refine(g, a, d, eps, 7 + r, part, level=0)
    rc, mp, st = pmo.map_graph(g, a, d, eps, 7, pmo.variants(repeats=3))
    assert st.levels == 1
    assert rc == rc_r and np.array_equal(mp, part) and st.j_final == st_r.j_final


@pytest.mark.parametrize("name", ["rgg14", "rmat14"])
def test_ultra_repeats_refinement_at_every_level(pmo, name):
    """Every run of Algorithm 6 has at least 12 loop bodies, so with R runs a
    level records at least 12 R; a second run from a run's own result never
    raises J (only strictly better feasible mappings replace the best)."""
    w = gen.get(name)
    g = w.graph()
    rc, part, st = pmo.map_graph(g, w.a, w.d, w.eps, 5, pmo.variants(repeats=4))
    assert all(st.level_iterations[s] >= 48 for s in range(st.levels))
    assert pmo.block_weights(g, part, w.k).max() <= st.lmax
    rc1, p1, s1 = pmo.refine(g, w.a, w.d, w.eps, 5, gen.random_balanced_mapping(g.n, w.k, 2))
    rc2, p2, s2 = pmo.refine(g, w.a, w.d, w.eps, 6, p1)
    assert s1.feasible and s2.feasible and s2.j_final <= s1.j_final


def test_ultra_hm_one_run_is_the_method(pmo):
    w = gen.get("rgg14")
    g = w.graph()
    rc0, p0 = pmo.hm(g, w.a, w.eps, 2)
    rc1, p1 = pmo.hm(g, w.a, w.eps, 2, pmo.variants(repeats=1))
    assert rc0 == rc1 and np.array_equal(p0, p1)
