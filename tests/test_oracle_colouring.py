"""Pins of the oracle's greedy colouring and colour-class ordering (not a
step of the paper: an ordering that bounds the depth of the ILU
substitutions of section "Iterative Solvers").  Closed forms on graphs whose
greedy colouring is known, the classic worst case of the greedy method, and
brute force on tiny graphs."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

import qsystems as qs
from oracle.liouvillian import liouvillian_sparse
from oracle.ordering import (colour_order, greedy_colouring, permute, random_visit, rcm, splitmix64,
                             symmetrized_pattern)
from oracle.transforms import modified, trace_population


def _graph(n, edges, loops=False):
    r = [a for a, b in edges] + [b for a, b in edges]
    c = [b for a, b in edges] + [a for a, b in edges]
    if loops:
        r += list(range(n))
        c += list(range(n))
    return sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(n, n))


def test_path_alternates_two_colours():
    n = 9
    col, k = greedy_colouring(_graph(n, [(i, i + 1) for i in range(n - 1)]), np.arange(n))
    assert k == 2 and col.tolist() == [i % 2 for i in range(n)]


def test_self_loops_are_not_edges():
    n = 7
    g = _graph(n, [(i, i + 1) for i in range(n - 1)], loops=True)
    col, k = greedy_colouring(g, np.arange(n))
    assert k == 2 and col.tolist() == [i % 2 for i in range(n)]


@pytest.mark.parametrize("n,k", [(6, 2), (7, 3)])
def test_cycle(n, k):
    col, used = greedy_colouring(_graph(n, [(i, (i + 1) % n) for i in range(n)]), np.arange(n))
    # 0, 1, 0, 1, ...; an odd cycle closes with a vertex next to both colours
    want = [i % 2 for i in range(n)]
    if n % 2:
        want[-1] = 2
    assert used == k and col.tolist() == want


def test_complete_graph_takes_the_visit_rank():
    n = 6
    order = np.array([3, 0, 5, 1, 4, 2])
    col, k = greedy_colouring(_graph(n, list(itertools.combinations(range(n), 2))), order)
    assert k == n and [col[v] for v in order] == list(range(n))


def test_star_depends_on_the_order():
    g = _graph(6, [(0, i) for i in range(1, 6)])
    col, k = greedy_colouring(g, np.arange(6))
    assert k == 2 and col.tolist() == [0, 1, 1, 1, 1, 1]
    col, k = greedy_colouring(g, np.array([1, 2, 3, 4, 5, 0]))
    assert k == 2 and col.tolist() == [1, 0, 0, 0, 0, 0]


@pytest.mark.parametrize("m", [2, 4, 6])
def test_crown_graph_worst_case(m):
    # K_{m,m} minus a perfect matching, visited a1 b1 a2 b2 ...: the greedy
    # method gives a_i and b_i colour i - 1 (m colours for a bipartite graph);
    # visiting one side first needs 2
    a, b = list(range(m)), list(range(m, 2 * m))
    g = _graph(2 * m, [(a[i], b[j]) for i in range(m) for j in range(m) if i != j])
    inter = np.array([x for i in range(m) for x in (a[i], b[i])])
    col, k = greedy_colouring(g, inter)
    assert k == m and col[a].tolist() == list(range(m)) and col[b].tolist() == list(range(m))
    col, k = greedy_colouring(g, np.arange(2 * m))
    assert k == min(m, 2) and set(col[a].tolist()) == {0}


def test_grid_row_major_is_a_checkerboard():
    R, C = 5, 7
    idx = lambda i, j: i * C + j
    edges = [(idx(i, j), idx(i, j + 1)) for i in range(R) for j in range(C - 1)]
    edges += [(idx(i, j), idx(i + 1, j)) for i in range(R - 1) for j in range(C)]
    col, k = greedy_colouring(_graph(R * C, edges), np.arange(R * C))
    assert k == 2 and all(col[idx(i, j)] == (i + j) % 2 for i in range(R) for j in range(C))


def _chromatic(n, edges):
    for k in range(1, n + 1):
        for c in itertools.product(range(k), repeat=n):
            if all(c[a] != c[b] for a, b in edges):
                return k
    return n


@pytest.mark.parametrize("seed", range(6))
def test_tiny_random_graphs_against_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = 7
    edges = [(a, b) for a, b in itertools.combinations(range(n), 2) if rng.random() < 0.45]
    order = rng.permutation(n)
    col, k = greedy_colouring(_graph(n, edges), order)
    deg = np.zeros(n, int)
    for a, b in edges:
        deg[a] += 1
        deg[b] += 1
        assert col[a] != col[b]
    assert _chromatic(n, edges) <= k <= deg.max() + 1
    rank = np.argsort(order)
    for v in range(n):
        earlier = {col[u] for a, b in edges for u, w in ((a, b), (b, a)) if w == v and rank[u] < rank[v]}
        # every smaller colour is blocked by an earlier neighbour
        assert set(range(col[v])) <= earlier and col[v] not in earlier


def test_order_rejects_a_non_permutation():
    with pytest.raises(ValueError):
        greedy_colouring(_graph(3, [(0, 1)]), np.array([0, 0, 1]))


def _depth_lower(A):
    A = sp.csr_matrix(A)
    lev = np.zeros(A.shape[0], dtype=np.int64)
    for i in range(A.shape[0]):
        c = A.indices[A.indptr[i]:A.indptr[i + 1]]
        c = c[c < i]
        lev[i] = lev[c].max() + 1 if c.size else 0
    return int(lev.max()) + 1


def test_splitmix64_published_outputs():
    # the first outputs of the reference generator seeded with 0
    assert [int(x) for x in splitmix64([0, 1, 2])] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                      0x06C45D188009454F]


def test_random_visit_is_the_priority_order():
    n = 5000
    order = random_visit(n)
    assert np.array_equal(np.sort(order), np.arange(n))
    pri = [int(x) for x in splitmix64(order)]
    assert all(a < b for a, b in zip(pri, pri[1:]))  # distinct here, so strictly increasing


@pytest.mark.parametrize("system", ["jc", "kerr_chain"])
def test_colour_order_on_liouvillians(system):
    s = qs.jaynes_cummings(6, seed=1) if system == "jc" else qs.kerr_chain(3, 3)
    L = liouvillian_sparse(s.H, s.c_ops)
    A, _, _ = modified(L, pop=trace_population(L))
    base = rcm(A)
    perm = colour_order(A)
    n = A.shape[0]
    assert np.array_equal(np.sort(perm), np.arange(n))
    col, k = greedy_colouring(symmetrized_pattern(A), random_visit(n))
    # classes in increasing colour, each in base order
    assert np.all(np.diff(col[perm]) >= 0)
    pos = np.empty(n, dtype=np.int64)
    pos[base] = np.arange(n)
    for c in range(k):
        cls = perm[col[perm] == c]
        assert np.all(np.diff(pos[cls]) > 0)
    # no off-diagonal entry inside a class, so the zero-fill lower factor has
    # at most k levels, far fewer than in RCM order
    B = permute(A, perm).tocoo()
    cp = col[perm]
    off = B.row != B.col
    assert np.all(cp[B.row[off]] != cp[B.col[off]])
    assert _depth_lower(permute(A, perm)) <= k < _depth_lower(permute(A, base))
