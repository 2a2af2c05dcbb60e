"""Pins for the oracle's SymCholesky (Section 3.2.3, Fig. 1)."""
import os

import numpy as np
import pytest

from oracle import symbolic as S

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fig1_cholesky_example.txt")


def _read_fig1():
    lower, factor, parent = {}, {}, None
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, rest = line.split(":", 1) if ":" in line else (line, "")
        vals = [int(v) for v in rest.split()]
        if key.startswith("matrix_lower"):
            lower[int(key.split()[1])] = vals
        elif key.startswith("factor"):
            factor[int(key.split()[1])] = vals
        elif key == "parent":
            parent = vals
    return lower, factor, parent


def _dense_symbolic(n, rows, cols):
    """Brute-force boolean elimination on a dense matrix: L pattern and etree."""
    M = np.zeros((n, n), dtype=bool)
    for i, j in zip(rows, cols):
        M[max(i, j), min(i, j)] = True
    M[np.arange(n), np.arange(n)] = True
    for k in range(n):
        below = np.nonzero(M[k + 1:, k])[0] + k + 1
        for a in below:
            for b in below:
                if b <= a:
                    M[a, b] = True
    parent = np.full(n, -1)
    for j in range(n):
        nz = np.nonzero(M[j + 1:, j])[0]
        if len(nz):
            parent[j] = j + 1 + nz[0]
    return M, parent


def test_fig1_etree_and_factor():
    lower, factor, parent = _read_fig1()
    rows = [r - 1 for c in lower for r in lower[c]]
    cols = [c - 1 for c in lower for r in lower[c]]
    colrows = S.permute_lower(rows, cols, np.arange(6))
    struct, par = S.column_structures(colrows)
    assert [p + 1 if p >= 0 else 0 for p in par] == parent
    for c in range(6):
        assert sorted(r + 1 for r in struct[c]) == factor[c + 1]
    counts = [len(s) for s in struct]
    assert counts == [3, 3, 3, 2, 2, 1]
    assert sum(counts) == 14 and len(rows) == 11
    # fill entries of panel (c) that panel (a) does not have
    fill = {(r + 1, c + 1) for c in range(6) for r in struct[c]} - {(r, c) for c in lower for r in lower[c]}
    assert fill == {(4, 3), (6, 3), (6, 4)}
    # natural order is already a postorder of this tree
    assert list(S.postorder(par)) == [0, 1, 2, 3, 4, 5]


def test_fig1_supernodes():
    lower, _, _ = _read_fig1()
    rows = [r - 1 for c in lower for r in lower[c]]
    cols = [c - 1 for c in lower for r in lower[c]]
    colrows = S.permute_lower(rows, cols, np.arange(6))
    struct, par = S.column_structures(colrows)
    cc = np.array([len(s) for s in struct])
    # (1-based) column 3 is the only child of column 4 and count(3) = count(4) + 1,
    # so {3, 4} is a fundamental supernode; 1, 2, 5, 6 stand alone
    assert S.fundamental_supernodes(par, cc) == [0, 1, 2, 4, 5]


@pytest.mark.parametrize("seed", range(12))
def test_structure_matches_dense_elimination(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 60))
    dens = rng.uniform(0.02, 0.2)
    rows, cols = [], []
    for i in range(n):
        for j in range(i):
            if rng.random() < dens:
                rows.append(i)
                cols.append(j)
    perm = rng.permutation(n)
    iperm = np.empty(n, dtype=int)
    iperm[perm] = np.arange(n)
    colrows = S.permute_lower(rows, cols, iperm)
    struct, par = S.column_structures(colrows)
    prow = [iperm[r] for r in rows]
    pcol = [iperm[c] for c in cols]
    M, par_dense = _dense_symbolic(n, prow, pcol)
    assert np.array_equal(par, par_dense)
    for j in range(n):
        assert sorted(struct[j]) == list(np.nonzero(M[:, j])[0])


@pytest.mark.parametrize("seed", range(12))
def test_liu_etree_matches_dense_elimination(seed):
    """The pattern-only elimination tree (Liu's algorithm) against brute-force
    boolean elimination of the permuted matrix."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(5, 80))
    dens = rng.uniform(0.02, 0.2)
    rows, cols = [], []
    for i in range(n):
        for j in range(i + 1):
            if i == j or rng.random() < dens:
                rows.append(i)
                cols.append(j)
    perm = rng.permutation(n)
    iperm = np.empty(n, dtype=int)
    iperm[perm] = np.arange(n)
    _, par_dense = _dense_symbolic(n, [iperm[r] for r in rows], [iperm[c] for c in cols])
    assert np.array_equal(S.etree_liu(n, rows, cols, iperm), par_dense)


def test_fig1_liu_etree():
    lower, _, parent = _read_fig1()
    rows = [r - 1 for c in lower for r in lower[c]]
    cols = [c - 1 for c in lower for r in lower[c]]
    par = S.etree_liu(6, rows, cols, np.arange(6))
    assert [p + 1 if p >= 0 else 0 for p in par] == parent


@pytest.mark.parametrize("G,H", [(4, 3), (8, 4), (12, 5)])
def test_final_permutation_equals_full_analysis(G, H):
    from oracle.plate import PlateOCP
    m = PlateOCP(G, H, 0.01)
    r, c = S.kkt_lower_pattern(m)
    a = S.analyze(m.n, r, c, lattice=(H, G, m.ns))
    assert np.array_equal(S.final_permutation(m.n, r, c, lattice=(H, G, m.ns)), a["perm"])


def _check_min_degree(n, rows, cols, order):
    """Replay elimination on a dense boolean adjacency matrix and check that each
    pivot had the minimum current degree, with ties broken by smallest index."""
    A = np.zeros((n, n), dtype=bool)
    for i, j in zip(rows, cols):
        if i != j:
            A[i, j] = A[j, i] = True
    alive = np.ones(n, dtype=bool)
    for v in order:
        deg = np.where(alive, (A & alive[None, :]).sum(axis=1), np.iinfo(np.int64).max)
        best = np.min(deg)
        assert deg[v] == best
        assert v == np.nonzero(deg == best)[0][0]
        nb = np.nonzero(A[v] & alive)[0]
        for a in nb:
            A[a, nb] = True
            A[a, a] = False
        alive[v] = False


@pytest.mark.parametrize("seed", range(8))
def test_min_degree_property(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(5, 50))
    rows, cols = [], []
    for i in range(n):
        for j in range(i):
            if rng.random() < 0.1:
                rows.append(i)
                cols.append(j)
    order = S.min_degree_order(n, S.adjacency_from_lower(n, rows, cols))
    assert sorted(order) == list(range(n))
    _check_min_degree(n, rows, cols, order)


def test_min_degree_small_graphs():
    # path 0-1-2-3-4: endpoints have degree 1; after 0 goes, 1 has degree 1 and wins the tie
    rows, cols = [1, 2, 3, 4], [0, 1, 2, 3]
    assert list(S.min_degree_order(5, S.adjacency_from_lower(5, rows, cols))) == [0, 1, 2, 3, 4]
    # star with centre 0 and leaves 1..5: leaves go first, then the centre ties with 5
    rows, cols = [1, 2, 3, 4, 5], [0, 0, 0, 0, 0]
    assert list(S.min_degree_order(6, S.adjacency_from_lower(6, rows, cols))) == [1, 2, 3, 4, 0, 5]


def test_analyze_invariants_distillation():
    from oracle.distillation import DistillationOCP
    m = DistillationOCP(6, 5, 0.1, 2.5)
    r, c = S.kkt_lower_pattern(m)
    a = S.analyze(m.n, r, c)
    n = m.n
    perm, iperm, par = a["perm"], a["iperm"], a["parent"]
    assert sorted(perm) == list(range(n))
    assert np.all(iperm[perm] == np.arange(n))
    # parent(j) > j, and the tree is postordered (every subtree is contiguous)
    assert all(par[j] > j or par[j] == -1 for j in range(n))
    first = np.arange(n)
    for j in range(n):
        if par[j] >= 0:
            first[par[j]] = min(first[par[j]], first[j])
    for j in range(n):
        assert np.all(par[first[j]:j] >= 0)
    # dense brute force on the permuted pattern gives the same factor pattern
    M, par_dense = _dense_symbolic(n, [iperm[i] for i in r], [iperm[j] for j in c])
    assert np.array_equal(par, par_dense)
    assert a["nnz_L"] == int(M.sum())
    # supernodes: contiguous cover; stored rows contain the exact structure of each column;
    # a child's rows below its columns are contained in its parent's rows
    sp_, rows_ = a["snode_ptr"], a["snode_rows"]
    assert sp_[0] == 0 and sp_[-1] == n and np.all(np.diff(sp_) > 0)
    for s in range(len(sp_) - 1):
        f, l = sp_[s], sp_[s + 1]
        R = set(rows_[s].tolist())
        assert list(rows_[s][:l - f]) == list(range(f, l))
        assert list(rows_[s]) == sorted(R)
        for j in range(f, l):
            assert set(np.nonzero(M[:, j])[0]) <= R
        p = a["snode_parent"][s]
        if p >= 0:
            assert set(rows_[s][l - f:].tolist()) <= set(rows_[p].tolist())
        else:
            assert len(rows_[s]) == l - f


@pytest.mark.parametrize("G,H", [(4, 3), (8, 4)])
def test_lattice_nested_dissection(G, H):
    """The plate's nested dissection is a permutation, its factor pattern equals
    brute-force dense elimination in that order, and it fills less than the
    stage-major natural order once the lattice is not tiny (the reason to
    dissect a 3-d lattice)."""
    from oracle.plate import PlateOCP
    m = PlateOCP(G, H, 0.01)
    r, c = S.kkt_lower_pattern(m)
    a = S.analyze(m.n, r, c, lattice=(H, G, m.ns))
    n, iperm = m.n, a["iperm"]
    assert sorted(a["perm"]) == list(range(n))
    M, par_dense = _dense_symbolic(n, [iperm[i] for i in r], [iperm[j] for j in c])
    assert np.array_equal(a["parent"], par_dense)
    assert a["nnz_L"] == int(M.sum())
    if G >= 8:   # on the smallest lattice the separators are most of the points
        Mn, _ = _dense_symbolic(n, list(r), list(c))
        assert a["nnz_L"] < int(Mn.sum())


def test_lattice_nested_dissection_top_separator():
    """A time cut of the stage lattice: with a slab of one stage the two halves
    share no matrix entry, so the slab's columns come last and the elimination
    tree has the two halves as separate subtrees below it."""
    from oracle.plate import PlateOCP
    G, H = 4, 7
    m = PlateOCP(G, H, 0.01)
    r, c = S.kkt_lower_pattern(m)
    adj = S.adjacency_from_lower(m.n, r, c)
    perm = S.lattice_nd_order(m.n, adj, H, G, m.ns)
    # box 7 x 4 x 4 = 112 points > leaf: time cut at 0 + (7 - 1) // 2 = 3 (16 points beat 2*7*4 = 56)
    slab = [3 * m.ns + p for p in range(G * G)]
    # the slab's points close the order, followed only by the controls no side holds alone
    tail = perm[len(perm) - len(slab) - 16:].tolist()
    assert set(slab) <= set(tail)
    assert all(v % m.ns >= G * G for v in tail if v not in slab)
    left = set(range(0, 3 * m.ns)) - set(slab)
    right = set(range(4 * m.ns, m.n))
    for i, j in zip(r, c):
        assert not ((i in left and j in right) or (i in right and j in left))


@pytest.mark.parametrize("N_,H", [(4, 7), (6, 12)])
def test_stage_nested_dissection(N_, H):
    """Stage nested dissection of the column: a permutation whose factor pattern
    equals dense elimination in that order; the middle stage separates the two
    halves (no matrix entry between them), and the elimination tree is shallow
    (its depth in columns is at most the separator stages times the stage size
    plus a leaf range)."""
    from oracle.distillation import DistillationOCP
    m = DistillationOCP(N_, H, 0.1, 2.5)
    r, c = S.kkt_lower_pattern(m)
    a = S.analyze(m.n, r, c, stages=(m.H, m.ns))
    n, iperm = m.n, a["iperm"]
    assert sorted(a["perm"]) == list(range(n))
    M, par_dense = _dense_symbolic(n, [iperm[i] for i in r], [iperm[j] for j in c])
    assert np.array_equal(a["parent"], par_dense)
    assert a["nnz_L"] == int(M.sum())
    order = S.stage_nd_order(H, m.ns)
    mid = (H - 1) // 2
    assert list(order[-m.ns:]) == list(range(mid * m.ns, (mid + 1) * m.ns))
    for i, j in zip(r, c):
        ti, tj = i // m.ns, j // m.ns
        assert not ((ti < mid < tj) or (tj < mid < ti))


def _check_cuts(cuts, r, c, ns):
    """No matrix entry joins the two sides of any cut over the cut's range."""
    side = {}
    for cut in cuts:
        if cut[0] == "time":
            _, t0, t1, V, pos = cut
            Vs = set(V)
            lo = {t * ns + v for t in range(t0, pos) for v in Vs}
            hi = {t * ns + v for t in range(pos + 1, t1) for v in Vs}
        else:
            _, t0, t1, left, sep, right = cut
            assert left and right and sep
            assert not (set(left) & set(right)) and not (set(sep) & (set(left) | set(right)))
            lo = {t * ns + v for t in range(t0, t1) for v in left}
            hi = {t * ns + v for t in range(t0, t1) for v in right}
        for i, j in zip(r, c):
            assert not ((i in lo and j in hi) or (i in hi and j in lo)), cut[:3]
        side[cut[:3]] = True
    return side


def test_graph_stage_nd_is_stage_nd_when_no_graph_cut_applies():
    """Small columns: every box either holds at most ND_LEAF points or is cut
    cheaper in time (a tray-chain level plus the two controls, which enter
    every tray's row, times the range), so the rule reduces to the stage
    nested dissection."""
    from oracle.distillation import DistillationOCP
    for N_, H in ((4, 7), (10, 20)):
        m = DistillationOCP(N_, H, 0.1, 2.5)
        r, c = S.kkt_lower_pattern(m)
        adj = S.adjacency_from_lower(m.n, r, c)
        cuts = []
        order = S.graph_stage_nd_order(m.n, adj, m.H, m.ns, m.nx, cuts=cuts)
        assert np.array_equal(order, S.stage_nd_order(m.H, m.ns))
        assert all(cut[0] == "time" for cut in cuts)


def test_graph_stage_nd_on_the_workload_column():
    """40 trays, horizon 100: short stage ranges are cut along the tray chain
    (a level of two trays plus both controls); every cut leaves its sides
    uncoupled and the factor is smaller than the stage nested dissection's."""
    from oracle.distillation import DistillationOCP
    m = DistillationOCP(40, 100, 0.05, 2.5)
    r, c = S.kkt_lower_pattern(m)
    adj = S.adjacency_from_lower(m.n, r, c)
    cuts = []
    S.graph_stage_nd_order(m.n, adj, m.H, m.ns, m.nx, cuts=cuts)
    _check_cuts(cuts, r, c, m.ns)
    graph = [cut for cut in cuts if cut[0] == "graph"]
    assert graph
    for cut in graph:       # the controls, where the box has them, are in the separator
        for u in (m.nx, m.nx + 1):
            assert u not in cut[3] and u not in cut[5]
    assert any(m.nx in cut[4] and m.nx + 1 in cut[4] for cut in graph)
    a = S.analyze(m.n, r, c, graph_stages=(m.H, m.ns, m.nx))
    b = S.analyze(m.n, r, c, stages=(m.H, m.ns))
    assert a["nnz_L"] < 0.7 * b["nnz_L"], (a["nnz_L"], b["nnz_L"])


@pytest.mark.parametrize("G,H", [(4, 3), (8, 6), (12, 1)])
def test_graph_stage_nd_on_the_plate(G, H):
    """On the plate's condensed matrix (whose stages are grids): a permutation;
    every cut, in time or in the graph, leaves its two sides uncoupled; graph
    cuts are made (the grid has long paths); the factor pattern equals dense
    elimination in that order; and the fill is below the stage nested
    dissection's (which keeps each stage whole) and within 10% of the lattice
    nested dissection's, which is told the grid (the heater controls follow
    the side of the nodes they heat, as there)."""
    from oracle.plate import PlateOCP
    m = PlateOCP(G, H, 0.01)
    r, c = S.kkt_lower_pattern(m)
    adj = S.adjacency_from_lower(m.n, r, c)
    cuts = []
    order = S.graph_stage_nd_order(m.n, adj, m.H, m.ns, m.nx, cuts=cuts)
    assert sorted(order.tolist()) == list(range(m.n))
    _check_cuts(cuts, r, c, m.ns)
    assert any(cut[0] == "graph" for cut in cuts)
    a = S.analyze(m.n, r, c, graph_stages=(m.H, m.ns, m.nx))
    iperm = a["iperm"]
    M, par_dense = _dense_symbolic(m.n, [iperm[i] for i in r], [iperm[j] for j in c])
    assert np.array_equal(a["parent"], par_dense)
    assert a["nnz_L"] == int(M.sum())
    b = S.analyze(m.n, r, c, stages=(m.H, m.ns))
    lat = S.analyze(m.n, r, c, lattice=(m.H, G, m.ns))
    if G >= 8:
        assert a["nnz_L"] < b["nnz_L"], (a["nnz_L"], b["nnz_L"])
        assert a["nnz_L"] <= 1.1 * lat["nnz_L"], (a["nnz_L"], lat["nnz_L"])


def test_graph_stage_nd_level_separator_on_a_path():
    """A single stage whose variables form a path 0 - 1 - ... - 99: the root
    search ends at an end of the path, the levels are single vertices, and
    the first cut takes the vertex where half the path is reached (every
    level in the balanced window has one vertex)."""
    n = 100
    adj = [set() for _ in range(n)]
    for v in range(n - 1):
        adj[v].add(v + 1)
        adj[v + 1].add(v)
    cuts = []
    order = S.graph_stage_nd_order(n, adj, 1, n, n, cuts=cuts)
    assert sorted(order.tolist()) == list(range(n))
    first = cuts[0]
    assert first[0] == "graph" and first[4] == [49]
    assert first[3] == list(range(49)) and first[5] == list(range(50, 100))
    assert order[-1] == 49
