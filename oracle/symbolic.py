"""SymCholesky on the CPU (oracle side), Section 3.2.3, eqs. (18)-(19), Fig. 1.

Given the lower-triangular sparsity pattern of the condensed matrix K_c^l
(diagonal included), compute

  * the fill-reducing permutation P (eq. 19).  The paper names minimum degree
    and nested dissection without fixing one.  The readings taken here: nested
    dissection of the stage structure by default -- the stage-and-graph
    nested dissection (rule below) for every family: stages couple only to
    their neighbours, so one stage separates the horizon (a shallow
    elimination tree, whose critical path is what a GPU factorization waits
    on), and within a range of stages a level of the graph the matrix
    induces on a stage's states separates it as well; the families' own
    dissections as an option -- stage nested dissection for the columns,
    lattice nested dissection for the plate family, whose condensed matrix
    is a three-dimensional (stage x grid) lattice -- and, as an option, exact
    minimum degree on the elimination graph (true degrees, no mass
    elimination, no absorption, no dense-row handling), ties broken by the
    smallest original index.  Every ordering is followed by a postorder of the
    elimination tree;
  * the elimination tree: parent(j) = min{ i > j : L_ij != 0 };
  * the column structures of L_P: struct(L_*j) = struct(K_P lower col j) united
    with struct(L_*c) minus {c} over the children c of j (Section 3.2.3);
  * fundamental supernodes and a relaxed amalgamation (rule below), which fix
    the stored pattern S_L including any explicit zeros.

Stage nested dissection.  A range [t0, t1) of stages with fewer than three
stages is ordered as is (increasing index); otherwise stage
pos = t0 + (t1 - t0 - 1) // 2 separates it: left range, right range, then the
variables of stage pos in increasing index.

Lattice nested dissection.  The variables of stage t are lattice points
(t, b, a) at index t ns + b G + a (a, b < G) followed by the stage's controls.
A box [t0, t1) x [b0, b1) x [a0, a1) of lattice points, with the controls
assigned to it, is ordered as follows.  If it holds at most ND_LEAF points, or
no dimension can be cut, its points in increasing index, then its controls in
increasing index.  Otherwise it is cut along one dimension by a separator slab
of thickness 1 in time (extent >= 3 needed) or 2 in space (extent >= 4
needed), since the condensed matrix couples stages only to their neighbours
and grid nodes up to two steps apart.  The dimension with the fewest separator
points wins, ties in the order time, b, a; the slab starts at
lo + (extent - thickness) // 2.  A control of the box goes to the left
(right) part if the lattice points it is coupled to in the matrix meet the
left (right) part only, otherwise to the separator.  Order: left box, right
box, the separator's points in increasing index, its controls in increasing
index.

Stage-and-graph nested dissection (models of the stage-pattern front end,
whose within-stage structure the analysis is not told).  With ns variables per
stage, nx of them states, the projected graph on [0, ns) joins a != b when the
matrix couples some variable a of one stage with variable b of the same or
another stage.  A box [t0, t1) x V (V a set of stage variables) has two
possible cuts:
  * in time, when t1 - t0 >= 3: stage pos = t0 + (t1 - t0 - 1) // 2 times V
    separates [t0, pos) x V from [pos + 1, t1) x V (|V| separator points);
  * in the graph, when (t1 - t0) |V| > ND_LEAF and V holds at least three
    states: a level structure of the projected graph restricted to V's
    states C (the levels of a breadth-first search: level 0 the root, level
    i + 1 the unvisited neighbours of level i).  The root: start at the
    smallest vertex of C; repeatedly take the vertex of the last level with
    the fewest neighbours in C (ties: smallest index) and move the root there
    while that lengthens the structure.  With L >= 3 levels and R states
    reached, the separator level l is, among the levels in [1, L - 2] whose
    predecessors hold between R / 4 and 3 R / 4 states, the smallest one
    (ties: levels 0..l holding closest to half of R, then the smallest l);
    with no such level, the smallest l in [1, L - 2] whose levels 0..l hold
    at least half of R, else L - 2.  The states of the levels before l form
    the left part, those after l and the unreached ones the right part.  A
    vertex of V that is not a state joins the left (right) part when its
    neighbours among C meet the left (right) part only, else the separator;
    then every such vertex with a neighbour across (left to right or right
    to left) moves to the separator, all at once.  ((t1 - t0) |separator|
    separator points.)  States of non-adjacent levels are never neighbours,
    so the two parts are uncoupled over the whole range.
The cut with fewer separator points wins, ties to the time cut; a box with no
cut lists its variables in increasing index.  Order: left box, right box, the
separator's variables in increasing index.  With no graph cut anywhere this is
the stage nested dissection.

Conventions: ``perm[k]`` is the original index of the k-th pivot (new -> old),
``iperm[v]`` is the pivot position of original index v (old -> new).

Relaxed amalgamation rule.  Supernodes are visited in increasing order of their
first column (a postorder of the supernodal tree).  A supernode s whose last
column's parent is the first column of the next supernode p (so s is the child
of p that immediately precedes it) is merged into p when
      width(s) + width(p) <= AMALG_MAX_WIDTH  and
      ( width(s) + width(p) <= AMALG_SMALL  or
        zeros(merged) <= AMALG_ZERO_FRAC * stored(merged) )
where stored(x) counts every entry a supernode stores in its trapezoid
(w (w + 1) / 2 + w * below) and zeros(x) counts explicit zeros, accumulated
over earlier merges.  A merged node keeps the later node's identity, so chains
of merges collapse bottom-up.
"""
from __future__ import annotations

import heapq
import numpy as np

ND_LEAF = 64
AMALG_MAX_WIDTH = 64
AMALG_SMALL = 8
AMALG_ZERO_FRAC = 0.25


def adjacency_from_lower(n, rows, cols):
    adj = [set() for _ in range(n)]
    for i, j in zip(rows, cols):
        i, j = int(i), int(j)
        if i != j:
            adj[i].add(j)
            adj[j].add(i)
    return adj


def min_degree_order(n, adj):
    """Exact minimum degree: returns perm (new -> old)."""
    adj = [set(a) for a in adj]
    heap = [(len(adj[v]), v) for v in range(n)]
    heapq.heapify(heap)
    done = [False] * n
    order = []
    while heap:
        d, v = heapq.heappop(heap)
        if done[v] or d != len(adj[v]):
            continue
        done[v] = True
        order.append(v)
        nb = adj[v]
        for a in nb:
            s = adj[a]
            s |= nb
            s.discard(a)
            s.discard(v)
            heapq.heappush(heap, (len(s), a))
        adj[v] = set()
    assert len(order) == n
    return np.array(order, dtype=np.int64)


def stage_nd_order(H, ns):
    """Stage nested dissection (rule in the module docstring): perm (new -> old)."""
    order = []

    def rec(t0, t1):
        if t1 - t0 < 3:
            order.extend(range(t0 * ns, t1 * ns))
            return
        pos = t0 + (t1 - t0 - 1) // 2
        rec(t0, pos)
        rec(pos + 1, t1)
        order.extend(range(pos * ns, (pos + 1) * ns))

    rec(0, H)
    return np.array(order, dtype=np.int64)


def _levels(adjV, V, root):
    """Breadth-first levels from root inside V (adjV: neighbours within V)."""
    seen = {root}
    levels = [[root]]
    while True:
        nxt = sorted({b for a in levels[-1] for b in adjV[a] if b not in seen})
        if not nxt:
            return levels
        seen.update(nxt)
        levels.append(nxt)


def graph_stage_nd_order(n, adj, H, ns, nx, cuts=None):
    """Stage-and-graph nested dissection (rule in the module docstring):
    perm (new -> old).  cuts, if a list, receives every cut made:
    ("time", t0, t1, V, pos) or ("graph", t0, t1, left, S, right)."""
    proj = [set() for _ in range(ns)]
    for i in range(n):
        for j in adj[i]:
            a, b = i % ns, j % ns
            if a != b:
                proj[a].add(b)
    order = []
    memo = {}    # a cut depends on V only, and time cuts repeat V over many ranges

    def graph_cut(V):
        key = tuple(V)
        if key not in memo:
            memo[key] = level_cut(V)
        return memo[key]

    def level_cut(V):
        C = [v for v in V if v < nx]
        if len(C) < 3:
            return None
        Cs = set(C)
        adjC = {a: [b for b in proj[a] if b in Cs] for a in C}
        lv = _levels(adjC, C, C[0])
        while True:
            cand = min(lv[-1], key=lambda v: (len(adjC[v]), v))
            lc = _levels(adjC, C, cand)
            if len(lc) > len(lv):
                lv = lc
            else:
                break
        L = len(lv)
        if L < 3:
            return None
        R = sum(len(x) for x in lv)
        before = [0] * L            # states in the levels before each level
        for l in range(1, L):
            before[l] = before[l - 1] + len(lv[l - 1])
        window = [l for l in range(1, L - 1) if R <= 4 * before[l] <= 3 * R]
        if window:
            sep = min(window, key=lambda l: (len(lv[l]), abs(2 * (before[l] + len(lv[l])) - R), l))
        else:
            sep = next((l for l in range(1, L - 1) if 2 * (before[l] + len(lv[l])) >= R), L - 2)
        left_states = {v for x in lv[:sep] for v in x}
        S = set(lv[sep])
        right_states = Cs - left_states - S
        left, right = set(left_states), set(right_states)
        for v in V:
            if v >= nx:
                inl = any(b in left_states for b in proj[v])
                inr = any(b in right_states for b in proj[v])
                (left if inl and not inr else right if inr and not inl else S).add(v)
        clash = {v for v in left if v >= nx and proj[v] & right} | {v for v in right if v >= nx and proj[v] & left}
        left -= clash
        right -= clash
        S |= clash
        return sorted(left), sorted(S), sorted(right)

    def emit(t0, t1, V):
        order.extend(t * ns + v for t in range(t0, t1) for v in V)

    def rec(t0, t1, V):
        best = None
        if t1 - t0 >= 3:
            best = (len(V), "time", None)
        if (t1 - t0) * len(V) > ND_LEAF:
            g = graph_cut(V)
            if g is not None and (best is None or (t1 - t0) * len(g[1]) < best[0]):
                best = ((t1 - t0) * len(g[1]), "graph", g)
        if best is None:
            emit(t0, t1, V)
            return
        if best[1] == "time":
            pos = t0 + (t1 - t0 - 1) // 2
            if cuts is not None:
                cuts.append(("time", t0, t1, list(V), pos))
            rec(t0, pos, V)
            rec(pos + 1, t1, V)
            emit(pos, pos + 1, V)
        else:
            left, S, right = best[2]
            if cuts is not None:
                cuts.append(("graph", t0, t1, left, S, right))
            rec(t0, t1, left)
            rec(t0, t1, right)
            emit(t0, t1, S)

    rec(0, H, list(range(ns)))
    if sorted(order) != list(range(n)):
        raise AssertionError("nested dissection did not produce a permutation")
    return np.array(order, dtype=np.int64)


def lattice_nd_order(n, adj, H, G, ns):
    """Lattice nested dissection (rule in the module docstring): perm (new -> old)."""
    nx = G * G

    def point(v):
        t, l = divmod(v, ns)
        return (t, l // G, l % G) if l < nx else None

    ctrl_pts = {}
    for t in range(H):
        for l in range(nx, ns):
            v = t * ns + l
            ctrl_pts[v] = [pt for pt in (point(u) for u in adj[v]) if pt is not None]

    def inside(pt, box):
        (t0, t1), (b0, b1), (a0, a1) = box
        return t0 <= pt[0] < t1 and b0 <= pt[1] < b1 and a0 <= pt[2] < a1

    def points(box):
        (t0, t1), (b0, b1), (a0, a1) = box
        return [t * ns + b * G + a for t in range(t0, t1) for b in range(b0, b1) for a in range(a0, a1)]

    order = []

    def rec(box, ctrls):
        ext = [hi - lo for lo, hi in box]
        vol = ext[0] * ext[1] * ext[2]
        cands = []
        if ext[0] >= 3:
            cands.append((ext[1] * ext[2], 0, 1))
        if ext[1] >= 4:
            cands.append((2 * ext[0] * ext[2], 1, 2))
        if ext[2] >= 4:
            cands.append((2 * ext[0] * ext[1], 2, 2))
        if vol <= ND_LEAF or not cands:
            order.extend(points(box))
            order.extend(sorted(ctrls))
            return
        _, dim, th = min(cands)
        lo, hi = box[dim]
        pos = lo + (hi - lo - th) // 2
        left = list(box); left[dim] = (lo, pos)
        sep = list(box); sep[dim] = (pos, pos + th)
        right = list(box); right[dim] = (pos + th, hi)
        cl, cr, cs = [], [], []
        for v in ctrls:
            inl = any(inside(pt, left) for pt in ctrl_pts[v])
            inr = any(inside(pt, right) for pt in ctrl_pts[v])
            (cl if inl and not inr else cr if inr and not inl else cs).append(v)
        rec(left, cl)
        rec(right, cr)
        order.extend(points(sep))
        order.extend(sorted(cs))

    rec([(0, H), (0, G), (0, G)], [t * ns + l for t in range(H) for l in range(nx, ns)])
    if sorted(order) != list(range(n)):
        raise AssertionError("nested dissection did not produce a permutation")
    return np.array(order, dtype=np.int64)


def permute_lower(rows, cols, iperm):
    """Lower pattern of P K P^T as per-column sorted row lists."""
    n = len(iperm)
    colrows = [set() for _ in range(n)]
    for i, j in zip(rows, cols):
        a, b = int(iperm[int(i)]), int(iperm[int(j)])
        if a < b:
            a, b = b, a
        colrows[b].add(a)
    for j in range(n):
        colrows[j].add(j)
    return colrows


def column_structures(colrows):
    """Column structures of L and the elimination tree, column by column.

    Children of j are the columns c < j with parent(c) = j; they are all known
    when column j is processed because parent(c) > c.
    """
    n = len(colrows)
    parent = np.full(n, -1, dtype=np.int64)
    struct = [None] * n
    children = [[] for _ in range(n)]
    for j in range(n):
        s = set(colrows[j])
        for c in children[j]:
            s |= struct[c]
        # drop the children themselves: every other row of a child's column is >= j
        s = {r for r in s if r >= j}
        struct[j] = s
        below = [r for r in s if r > j]
        if below:
            p = min(below)
            parent[j] = p
            children[p].append(j)
    return struct, parent


def postorder(parent):
    """DFS postorder; roots and children visited in increasing index."""
    n = len(parent)
    children = [[] for _ in range(n)]
    roots = []
    for j in range(n):
        if parent[j] < 0:
            roots.append(j)
        else:
            children[parent[j]].append(j)
    post = []
    for r in roots:
        stack = [(r, 0)]
        while stack:
            v, ci = stack.pop()
            if ci < len(children[v]):
                stack.append((v, ci + 1))
                stack.append((children[v][ci], 0))
            else:
                post.append(v)
    return np.array(post, dtype=np.int64)


def fundamental_supernodes(parent, colcount):
    """Column j+1 joins j's supernode iff parent(j) = j+1, j is the only child
    of j+1, and colcount(j) = colcount(j+1) + 1.  Returns supernode start list."""
    n = len(parent)
    nchild = np.zeros(n, dtype=np.int64)
    for j in range(n):
        if parent[j] >= 0:
            nchild[parent[j]] += 1
    starts = [0]
    for j in range(n - 1):
        same = (parent[j] == j + 1 and nchild[j + 1] == 1
                and colcount[j] == colcount[j + 1] + 1)
        if not same:
            starts.append(j + 1)
    return starts


def amalgamate(starts, parent, struct, n):
    """Relaxed amalgamation (rule in the module docstring)."""
    nodes = []   # each: [first, last_excl, below_rows(set), stored, zeros]
    bounds = list(starts) + [n]
    for s in range(len(starts)):
        f, l = bounds[s], bounds[s + 1]
        below = {r for r in struct[f] if r >= l}
        w = l - f
        stored = w * (w + 1) // 2 + w * len(below)
        nodes.append([f, l, below, stored, 0])
    out = []
    for node in nodes:
        # try to merge the previously emitted node (immediately preceding) into this one
        while out:
            prev = out[-1]
            f0, l0 = prev[0], prev[1]
            if l0 != node[0] or parent[l0 - 1] != node[0]:
                break
            w = node[1] - prev[0]
            below = node[2]
            stored = w * (w + 1) // 2 + w * len(below)
            zeros = stored - (prev[3] - prev[4]) - (node[3] - node[4])
            ok = w <= AMALG_MAX_WIDTH and (w <= AMALG_SMALL or zeros <= AMALG_ZERO_FRAC * stored)
            if not ok:
                break
            out.pop()
            node = [prev[0], node[1], below, stored, zeros]
        out.append(node)
    snode_ptr = np.array([nd[0] for nd in out] + [n], dtype=np.int64)
    rows = []
    for nd in out:
        rows.append(np.array(list(range(nd[0], nd[1])) + sorted(nd[2]), dtype=np.int64))
    return snode_ptr, rows


def etree_liu(n, rows, cols, iperm):
    """Elimination tree of P K P^T straight from the pattern (Liu's algorithm
    with path compression; no column structures), for sizes where the column
    structures of L do not fit in memory.  rows/cols: lower pattern in the
    original indexing; iperm: old -> new.  parent(j) = min{i > j : L_ij != 0}:
    row k of the permuted matrix is visited in increasing k; from every
    earlier column i it touches, the walk climbs i's current ancestors to the
    root of i's subtree, which becomes a child of k."""
    a = np.asarray(iperm, dtype=np.int64)[np.asarray(rows, dtype=np.int64)]
    b = np.asarray(iperm, dtype=np.int64)[np.asarray(cols, dtype=np.int64)]
    hi, lo = np.maximum(a, b), np.minimum(a, b)
    off = hi != lo
    hi, lo = hi[off], lo[off]
    order = np.lexsort((lo, hi))
    hi, lo = hi[order].tolist(), lo[order].tolist()
    parent = [-1] * n
    anc = [-1] * n
    for k, i in zip(hi, lo):
        while True:
            nxt = anc[i]
            anc[i] = k
            if nxt == -1:
                parent[i] = k
                break
            if nxt == k:
                break
            i = nxt
    return np.array(parent, dtype=np.int64)


def final_permutation(n, rows, cols, lattice=None, stages=None, graph_stages=None):
    """The permutation of ``analyze`` (ordering, then the postorder of its
    elimination tree) without the column structures: perm (new -> old)."""
    if lattice is not None:
        perm_md = lattice_nd_order(n, adjacency_from_lower(n, rows, cols), *lattice)
    elif graph_stages is not None:
        perm_md = graph_stage_nd_order(n, adjacency_from_lower(n, rows, cols), *graph_stages)
    elif stages is not None:
        perm_md = stage_nd_order(*stages)
    else:
        perm_md = min_degree_order(n, adjacency_from_lower(n, rows, cols))
    iperm_md = np.empty(n, dtype=np.int64)
    iperm_md[perm_md] = np.arange(n)
    return perm_md[postorder(etree_liu(n, rows, cols, iperm_md))]


def analyze(n, rows, cols, lattice=None, stages=None, graph_stages=None):
    """Full symbolic analysis of a lower pattern (original indexing).

    lattice = (H, G, ns) selects the lattice nested dissection of a plate
    transcription, stages = (H, ns) the stage nested dissection of a
    stage-major transcription, graph_stages = (H, ns, nx) the stage-and-graph
    nested dissection; otherwise exact minimum degree.  Returns a dict with perm,
    iperm, parent (column etree in final order), colcount (per column of the
    exact factor), nnz_L (exact), snode_ptr, snode_rows (row list per supernode,
    stored pattern), snode_parent.
    """
    adj = adjacency_from_lower(n, rows, cols)
    if lattice is not None:
        perm_md = lattice_nd_order(n, adj, *lattice)
    elif graph_stages is not None:
        perm_md = graph_stage_nd_order(n, adj, *graph_stages)
    elif stages is not None:
        perm_md = stage_nd_order(*stages)
    else:
        perm_md = min_degree_order(n, adj)
    iperm_md = np.empty(n, dtype=np.int64)
    iperm_md[perm_md] = np.arange(n)
    colrows = permute_lower(rows, cols, iperm_md)
    _, parent_md = column_structures(colrows)
    post = postorder(parent_md)
    perm = perm_md[post]
    iperm = np.empty(n, dtype=np.int64)
    iperm[perm] = np.arange(n)
    colrows = permute_lower(rows, cols, iperm)
    struct, parent = column_structures(colrows)
    colcount = np.array([len(s) for s in struct], dtype=np.int64)
    starts = fundamental_supernodes(parent, colcount)
    snode_ptr, snode_rows = amalgamate(starts, parent, struct, n)
    nsn = len(snode_ptr) - 1
    col2sn = np.empty(n, dtype=np.int64)
    for s in range(nsn):
        col2sn[snode_ptr[s]:snode_ptr[s + 1]] = s
    snode_parent = np.full(nsn, -1, dtype=np.int64)
    for s in range(nsn):
        last = snode_ptr[s + 1] - 1
        if parent[last] >= 0:
            snode_parent[s] = col2sn[parent[last]]
    return dict(n=n, perm=perm, iperm=iperm, parent=parent, colcount=colcount,
                nnz_L=int(colcount.sum()), flops=int(np.sum(colcount.astype(np.int64) ** 2)),
                snode_ptr=snode_ptr, snode_rows=snode_rows, snode_parent=snode_parent,
                struct=struct, colrows=colrows)


def kkt_lower_pattern(nlp):
    """Structural lower pattern of K = W + J_c^T J_c + J_d^T J_d + diag (original order)."""
    import scipy.sparse as sp
    n = nlp.n
    ent = set()
    for r, c in zip(nlp.h_rows, nlp.h_cols):
        ent.add((max(r, c), min(r, c)))
    for rows_, cols_, m in ((nlp.jc_rows, nlp.jc_cols, nlp.m_c), (nlp.jd_rows, nlp.jd_cols, nlp.m_d)):
        if m == 0:
            continue
        J = sp.csr_matrix((np.ones(len(rows_)), (rows_, cols_)), shape=(m, n))
        for r in range(m):
            cs = J.indices[J.indptr[r]:J.indptr[r + 1]]
            for a in cs:
                for b in cs:
                    if a >= b:
                        ent.add((int(a), int(b)))
    for j in range(n):
        ent.add((j, j))
    ent = sorted(ent, key=lambda t: (t[1], t[0]))
    return np.array([e[0] for e in ent]), np.array([e[1] for e in ent])
