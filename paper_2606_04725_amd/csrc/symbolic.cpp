// SymCholesky on the host (Section 3.2.3, eqs. 18-19, Fig. 1), computed once
// per problem structure and reused by every numeric factorization.
//
//  1. Fill-reducing ordering P (NMPC_ORDER_* of the structure).  Minimum
//     degree: exact, on the elimination graph of the condensed matrix pattern
//     (true degrees, no mass elimination, no element absorption; ties go to the
//     smallest original index).  Family dissection: for the
//     distillation families (the workload column and the reflux column of the
//     case study) and front-end models by stages (a range of fewer than three stages keeps
//     its order, otherwise its middle stage t0 + (t1 - t0 - 1) / 2 separates
//     it: left range, right range, separator stage); for the plate family on
//     the (stage x grid) lattice of its condensed matrix: a box of lattice
//     points is cut by a slab one stage thick or two grid lines thick (the
//     matrix couples neighbouring stages and nodes up to two steps apart),
//     along the dimension with the fewest slab points (ties: time, row,
//     column), the slab starting at lo + (extent - thickness) / 2; boxes of at
//     most kNdLeaf points, or with no cuttable dimension, are leaves.  A control
//     follows the side holding every lattice point it is coupled to, else the
//     slab.  Order: left box, right box, slab points, slab controls; inside a
//     leaf, points then controls, each in increasing index.  Nested
//     dissection, the default for every family, on the (stage x projected
//     graph) product of the condensed matrix, which needs no geometry (the
//     first nx variables of a stage are its states): the projected graph joins stage
//     variables a != b that the matrix couples in any pair of stages; a box
//     [t0, t1) x V is cut in time (t1 - t0 >= 3: the middle stage t0 +
//     (t1 - t0 - 1) / 2 times V) or, when it holds more than kNdLeaf points
//     and V at least 3 states, in the graph by one level of a breadth-first
//     level structure over V's states (root moved from the smallest state to
//     the least-connected state of the last level while that lengthens the
//     structure; with L >= 3 levels and R states reached: among levels l in
//     [1, L - 2] with between R / 4 and 3 R / 4 states before them the
//     smallest, ties closest to halving R, then the first; none: the first
//     level whose prefix holds half of R, else L - 2).  Earlier levels go
//     left, later levels and unreached states right; a non-state joins the
//     side its state neighbours lie on when they lie on one side, else the
//     separator, and non-states with a neighbour across the cut then move to
//     the separator together.  Fewer separator points wins, ties to time; no
//     cut: the box's variables in increasing index.
//  2. Elimination tree parent(j) = min{i > j : L_ij != 0} and column
//     structures struct(L_*j) = struct(K_P lower col j) united with the
//     structures of j's children minus the children themselves.
//  3. Postorder (children and roots in increasing index) composed into P, then
//     step 2 again in the final order.
//  4. Fundamental supernodes, then relaxed amalgamation: walking supernodes in
//     order, the immediately preceding node is merged into the current one
//     when it is that node's child, the merged width is at most 64, and the
//     merged width is at most 8 or its explicit zeros are at most a quarter of
//     its stored entries.
//  5. Maps for the numeric phase: factor-order KKT slots with their position in
//     the supernode front, the J^T Q J contributions of each slot, relative
//     row positions of every child's update block inside its parent, and a
//     bottom-up level schedule of the supernodal tree.
#include <algorithm>
#include <cstdint>
#include <map>
#include <queue>
#include <stdexcept>
#include <utility>

#include "internal.h"

namespace nmpc {

namespace {

constexpr int kAmalgMaxWidth = 64;
constexpr int kNdLeaf = 64;
constexpr int kAmalgSmall = 8;

using Adj = std::vector<std::vector<int32_t>>;

void sorted_insert_union(std::vector<int32_t>& dst, const std::vector<int32_t>& src) {
    std::vector<int32_t> out;
    out.reserve(dst.size() + src.size());
    std::set_union(dst.begin(), dst.end(), src.begin(), src.end(), std::back_inserter(out));
    dst.swap(out);
}

void erase_sorted(std::vector<int32_t>& v, int32_t x) {
    auto it = std::lower_bound(v.begin(), v.end(), x);
    if (it != v.end() && *it == x) v.erase(it);
}

// Exact minimum degree (returns perm, new -> old).
std::vector<int32_t> min_degree(int n, Adj adj) {
    using Item = std::pair<int64_t, int32_t>;   // (degree, vertex); min-heap
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
    for (int v = 0; v < n; ++v) heap.push({(int64_t)adj[v].size(), v});
    std::vector<char> done(n, 0);
    std::vector<int32_t> order;
    order.reserve(n);
    while (!heap.empty()) {
        auto [d, v] = heap.top();
        heap.pop();
        if (done[v] || d != (int64_t)adj[v].size()) continue;
        done[v] = 1;
        order.push_back(v);
        const std::vector<int32_t> nb = adj[v];
        for (int32_t a : nb) {
            sorted_insert_union(adj[a], nb);
            erase_sorted(adj[a], a);
            erase_sorted(adj[a], v);
            heap.push({(int64_t)adj[a].size(), a});
        }
        adj[v].clear();
        adj[v].shrink_to_fit();
    }
    if ((int)order.size() != n) throw std::runtime_error("minimum degree: incomplete order");
    return order;
}

// Lattice nested dissection of a stage-major (stage x G x G grid) + controls
// transcription (returns perm, new -> old).
struct NdBox {
    int lo[3], hi[3];   // stage, grid row b, grid column a
};

class LatticeNd {
  public:
    LatticeNd(int n, int H, int G, int ns, const std::vector<std::pair<int32_t, int32_t>>& ent)
        : n_(n), H_(H), G_(G), ns_(ns), nx_(G * G), pts_(n) {
        for (auto [i, j] : ent) {
            if (i == j) continue;
            if (is_ctrl(i) && !is_ctrl(j)) pts_[i].push_back(j);
            if (is_ctrl(j) && !is_ctrl(i)) pts_[j].push_back(i);
        }
    }
    std::vector<int32_t> order() {
        std::vector<int32_t> ctrls;
        for (int v = 0; v < n_; ++v)
            if (is_ctrl(v)) ctrls.push_back(v);
        NdBox b{{0, 0, 0}, {H_, G_, G_}};
        out_.clear();
        out_.reserve(n_);
        rec(b, ctrls);
        return out_;
    }

  private:
    bool is_ctrl(int v) const { return v % ns_ >= nx_; }
    bool inside(int v, const NdBox& b) const {
        const int t = v / ns_, l = v % ns_, r = l / G_, c = l % G_;
        return t >= b.lo[0] && t < b.hi[0] && r >= b.lo[1] && r < b.hi[1] && c >= b.lo[2] && c < b.hi[2];
    }
    void emit_points(const NdBox& b) {
        for (int t = b.lo[0]; t < b.hi[0]; ++t)
            for (int r = b.lo[1]; r < b.hi[1]; ++r)
                for (int c = b.lo[2]; c < b.hi[2]; ++c) out_.push_back(t * ns_ + r * G_ + c);
    }
    void rec(const NdBox& b, std::vector<int32_t>& ctrls) {
        const int64_t e0 = b.hi[0] - b.lo[0], e1 = b.hi[1] - b.lo[1], e2 = b.hi[2] - b.lo[2];
        int64_t best = -1;
        int dim = -1, th = 0;
        auto consider = [&](int64_t size, int d, int t) {
            if (best < 0 || size < best) {
                best = size;
                dim = d;
                th = t;
            }
        };
        if (e0 >= 3) consider(e1 * e2, 0, 1);
        if (e1 >= 4) consider(2 * e0 * e2, 1, 2);
        if (e2 >= 4) consider(2 * e0 * e1, 2, 2);
        if (e0 * e1 * e2 <= kNdLeaf || dim < 0) {
            emit_points(b);
            std::sort(ctrls.begin(), ctrls.end());
            out_.insert(out_.end(), ctrls.begin(), ctrls.end());
            return;
        }
        const int lo = b.lo[dim], hi = b.hi[dim];
        const int pos = lo + (hi - lo - th) / 2;
        NdBox left = b, sep = b, right = b;
        left.hi[dim] = pos;
        sep.lo[dim] = pos;
        sep.hi[dim] = pos + th;
        right.lo[dim] = pos + th;
        std::vector<int32_t> cl, cr, cs;
        for (int32_t v : ctrls) {
            bool inl = false, inr = false;
            for (int32_t q : pts_[v]) {
                inl = inl || inside(q, left);
                inr = inr || inside(q, right);
            }
            (inl && !inr ? cl : (inr && !inl ? cr : cs)).push_back(v);
        }
        rec(left, cl);
        rec(right, cr);
        emit_points(sep);
        std::sort(cs.begin(), cs.end());
        out_.insert(out_.end(), cs.begin(), cs.end());
    }
    int n_, H_, G_, ns_, nx_;
    std::vector<std::vector<int32_t>> pts_;   // lattice points coupled to each control
    std::vector<int32_t> out_;
};

// Stage nested dissection of a stage-major transcription (perm, new -> old).
std::vector<int32_t> stage_nd(int H, int ns) {
    std::vector<int32_t> out;
    out.reserve((size_t)H * ns);
    struct Frame {   // a range of stages and how far its order has got
        int t0, t1, state;
    };
    std::vector<Frame> st{{0, H, 0}};
    while (!st.empty()) {
        Frame& f = st.back();
        if (f.t1 - f.t0 < 3) {
            for (int v = f.t0 * ns; v < f.t1 * ns; ++v) out.push_back(v);
            st.pop_back();
            continue;
        }
        const int pos = f.t0 + (f.t1 - f.t0 - 1) / 2;
        if (f.state == 0) {
            f.state = 1;
            st.push_back({f.t0, pos, 0});
        } else if (f.state == 1) {
            f.state = 2;
            st.push_back({pos + 1, f.t1, 0});
        } else {
            for (int v = pos * ns; v < (pos + 1) * ns; ++v) out.push_back(v);
            st.pop_back();
        }
    }
    return out;
}

// Stage-and-graph nested dissection of a stage-major transcription whose
// stages carry no geometry (perm, new -> old); ent: lower pattern entries;
// the first nx variables of a stage are its states.
class GraphStageNd {
  public:
    GraphStageNd(int n, int H, int ns, int nx, const std::vector<std::pair<int32_t, int32_t>>& ent)
        : H_(H), ns_(ns), nx_(nx), proj_(ns), in_(ns, 0), seen_(ns, 0), side_(ns, 0) {
        for (auto [i, j] : ent) {
            const int a = i % ns, b = j % ns;
            if (i != j && a != b) {
                proj_[a].push_back(b);
                proj_[b].push_back(a);
            }
        }
        for (auto& l : proj_) {
            std::sort(l.begin(), l.end());
            l.erase(std::unique(l.begin(), l.end()), l.end());
        }
        out_.reserve(n);
    }
    std::vector<int32_t> order() {
        std::vector<int32_t> all(ns_);
        for (int v = 0; v < ns_; ++v) all[v] = v;
        rec(0, H_, all);
        return out_;
    }

  private:
    using Levels = std::vector<std::vector<int32_t>>;
    // breadth-first levels from root inside the states marked with stamp_in_
    Levels levels(int32_t root) {
        const int s = ++stamp_seen_;
        Levels lv{{root}};
        seen_[root] = s;
        for (;;) {
            std::vector<int32_t> nxt;
            for (int32_t a : lv.back())
                for (int32_t b : proj_[a])
                    if (in_[b] == stamp_in_ && seen_[b] != s) {
                        seen_[b] = s;
                        nxt.push_back(b);
                    }
            if (nxt.empty()) return lv;
            std::sort(nxt.begin(), nxt.end());
            lv.push_back(std::move(nxt));
        }
    }
    int deg_in(int32_t v) const {
        int d = 0;
        for (int32_t b : proj_[v]) d += in_[b] == stamp_in_;
        return d;
    }
    // level-structure cut of V over its states: false when V holds fewer than
    // 3 states or their structure has fewer than 3 levels
    bool graph_cut(const std::vector<int32_t>& V, std::vector<int32_t>& left, std::vector<int32_t>& sep,
                   std::vector<int32_t>& right) {
        stamp_in_ = ++stamp_in_ctr_;
        int nc = 0;
        int32_t first = -1;
        for (int32_t v : V)
            if (v < nx_) {
                in_[v] = stamp_in_;
                if (first < 0) first = v;
                ++nc;
            }
        if (nc < 3) return false;
        Levels lv = levels(first);
        for (;;) {
            int32_t cand = -1;
            int cdeg = 0;
            for (int32_t v : lv.back()) {
                const int d = deg_in(v);
                if (cand < 0 || d < cdeg || (d == cdeg && v < cand)) {
                    cand = v;
                    cdeg = d;
                }
            }
            Levels lc = levels(cand);
            if (lc.size() > lv.size()) lv = std::move(lc);
            else break;
        }
        const int L = (int)lv.size();
        if (L < 3) return false;
        std::vector<int64_t> before(L, 0);   // states in the levels before each level
        for (int l = 1; l < L; ++l) before[l] = before[l - 1] + (int64_t)lv[l - 1].size();
        const int64_t R = before[L - 1] + (int64_t)lv[L - 1].size();
        int cut = -1;
        int64_t csize = 0, cdist = 0;
        for (int l = 1; l <= L - 2; ++l) {
            if (4 * before[l] < R || 4 * before[l] > 3 * R) continue;
            const int64_t sz = (int64_t)lv[l].size();
            const int64_t dist = std::llabs(2 * (before[l] + sz) - R);
            if (cut < 0 || sz < csize || (sz == csize && dist < cdist)) {
                cut = l;
                csize = sz;
                cdist = dist;
            }
        }
        if (cut < 0) {
            cut = L - 2;
            for (int l = 1; l <= L - 2; ++l)
                if (2 * (before[l] + (int64_t)lv[l].size()) >= R) {
                    cut = l;
                    break;
                }
        }
        // sides: 1 left, 2 separator, 3 right (states first, then the others)
        const int base = stamp_side_ += 4;
        for (int l = 0; l < L; ++l)
            for (int32_t v : lv[l]) side_[v] = base + (l < cut ? 1 : (l == cut ? 2 : 3));
        for (int32_t v : V)
            if (v < nx_ && (side_[v] <= base || side_[v] > base + 3)) side_[v] = base + 3;   // unreached
        for (int32_t v : V) {
            if (v < nx_) continue;
            bool inl = false, inr = false;
            for (int32_t b : proj_[v])
                if (b < nx_ && in_[b] == stamp_in_) {
                    inl = inl || side_[b] == base + 1;
                    inr = inr || side_[b] == base + 3;
                }
            side_[v] = base + (inl && !inr ? 1 : (inr && !inl ? 3 : 2));
        }
        // non-states with a neighbour across the cut move to the separator, all at once
        std::vector<int32_t> clash;
        for (int32_t v : V) {
            if (v < nx_ || side_[v] == base + 2) continue;
            const int other = side_[v] == base + 1 ? base + 3 : base + 1;
            for (int32_t b : proj_[v])   // (vertices outside V hold older stamps)
                if (side_[b] == other) {
                    clash.push_back(v);
                    break;
                }
        }
        for (int32_t v : clash) side_[v] = base + 2;
        left.clear();
        sep.clear();
        right.clear();
        for (int32_t v : V) (side_[v] == base + 1 ? left : (side_[v] == base + 2 ? sep : right)).push_back(v);
        return true;
    }
    void emit(int t0, int t1, const std::vector<int32_t>& V) {
        for (int t = t0; t < t1; ++t)
            for (int32_t v : V) out_.push_back(t * ns_ + v);
    }
    void rec(int t0, int t1, const std::vector<int32_t>& V) {
        const int64_t span = t1 - t0;
        bool have = false, graph = false;
        int64_t best = 0;
        if (span >= 3) {
            have = true;
            best = (int64_t)V.size();
        }
        std::vector<int32_t> left, sep, right;
        if (span * (int64_t)V.size() > kNdLeaf && graph_cut(V, left, sep, right) &&
            (!have || span * (int64_t)sep.size() < best)) {
            have = graph = true;
        }
        if (!have) {
            emit(t0, t1, V);
        } else if (!graph) {
            const int pos = t0 + (t1 - t0 - 1) / 2;
            rec(t0, pos, V);
            rec(pos + 1, t1, V);
            emit(pos, pos + 1, V);
        } else {
            rec(t0, t1, left);
            rec(t0, t1, right);
            emit(t0, t1, sep);
        }
    }
    int H_, ns_, nx_;
    std::vector<std::vector<int32_t>> proj_;
    std::vector<int> in_, seen_, side_;
    int stamp_in_ = 0, stamp_in_ctr_ = 0, stamp_seen_ = 0, stamp_side_ = 0;
    std::vector<int32_t> out_;
};

// Lower pattern of P K P^T as sorted per-column row lists (diagonal included).
Adj permute_lower(int n, const std::vector<std::pair<int32_t, int32_t>>& ent,
                  const std::vector<int32_t>& iperm) {
    Adj col(n);
    for (auto [i, j] : ent) {
        int a = iperm[i], b = iperm[j];
        if (a < b) std::swap(a, b);
        col[b].push_back(a);
    }
    for (int j = 0; j < n; ++j) {
        col[j].push_back(j);
        std::sort(col[j].begin(), col[j].end());
        col[j].erase(std::unique(col[j].begin(), col[j].end()), col[j].end());
    }
    return col;
}

// Column structures of L and the elimination tree.
void column_structures(const Adj& colrows, Adj& strct, std::vector<int32_t>& parent) {
    const int n = (int)colrows.size();
    strct.assign(n, {});
    parent.assign(n, -1);
    std::vector<std::vector<int32_t>> children(n);
    for (int j = 0; j < n; ++j) {
        std::vector<int32_t> s = colrows[j];
        for (int32_t c : children[j]) {
            std::vector<int32_t> t(strct[c].begin() + 1, strct[c].end());  // drop c itself
            sorted_insert_union(s, t);
        }
        // every row is >= j: colrows has rows >= j, children's rows beyond c are >= j
        strct[j] = std::move(s);
        if (strct[j].size() > 1) {
            parent[j] = strct[j][1];
            children[parent[j]].push_back(j);
        }
    }
}

std::vector<int32_t> postorder(const std::vector<int32_t>& parent) {
    const int n = (int)parent.size();
    std::vector<std::vector<int32_t>> children(n);
    std::vector<int32_t> roots;
    for (int j = 0; j < n; ++j) {
        if (parent[j] < 0) roots.push_back(j);
        else children[parent[j]].push_back(j);
    }
    std::vector<int32_t> post;
    post.reserve(n);
    std::vector<std::pair<int32_t, size_t>> stack;
    for (int32_t r : roots) {
        stack.push_back({r, 0});
        while (!stack.empty()) {
            auto& top = stack.back();
            if (top.second < children[top.first].size()) {
                int32_t c = children[top.first][top.second++];
                stack.push_back({c, 0});
            } else {
                post.push_back(top.first);
                stack.pop_back();
            }
        }
    }
    return post;
}

struct SNode {
    int32_t f, l;
    std::vector<int32_t> below;
    int64_t stored, zeros;
};

}  // namespace

// Offsets of the update blocks ((rows - width)^2 doubles each) in a pool where
// a block lives from its supernode's execution level until its parent's level
// has run; released blocks are reused best-fit.  lev[s] is the step at which
// supernode s runs: every supernode of a step must finish before the next step
// starts, or a reused block could still be in use.
void update_block_pool(const Symbolic& sym, const std::vector<int>& lev, std::vector<int64_t>& u_off,
                       int64_t& stored_u) {
    const int nsn = (int)sym.sn_ptr.size() - 1;
    int depth = 0;
    for (int s = 0; s < nsn; ++s) depth = std::max(depth, lev[s] + 1);
    u_off.assign(nsn + 1, 0);
    std::vector<std::vector<int32_t>> born(depth + 1), freed(depth + 2);
    for (int s = 0; s < nsn; ++s) {
        born[lev[s]].push_back(s);
        const int end = sym.sn_parent[s] >= 0 ? lev[sym.sn_parent[s]] : lev[s];
        freed[end + 1].push_back(s);
    }
    std::map<int64_t, int64_t> holes;   // offset -> size
    int64_t top = 0;
    auto ublock = [&](int s) {
        const int64_t w = sym.sn_ptr[s + 1] - sym.sn_ptr[s];
        const int64_t mr = sym.sn_rows_ptr[s + 1] - sym.sn_rows_ptr[s];
        return (mr - w) * (mr - w);
    };
    for (int L = 0; L <= depth; ++L) {
        for (int32_t s : freed[L]) {
            const int64_t sz = ublock(s);
            if (sz == 0) continue;
            auto it = holes.emplace(u_off[s], sz).first;
            auto nx = std::next(it);
            if (nx != holes.end() && it->first + it->second == nx->first) {
                it->second += nx->second;
                holes.erase(nx);
            }
            if (it != holes.begin()) {
                auto pv = std::prev(it);
                if (pv->first + pv->second == it->first) {
                    pv->second += it->second;
                    holes.erase(it);
                }
            }
        }
        if (L == depth) break;
        for (int32_t s : born[L]) {
            const int64_t sz = ublock(s);
            if (sz == 0) {
                u_off[s] = 0;
                continue;
            }
            auto best = holes.end();
            for (auto it = holes.begin(); it != holes.end(); ++it)
                if (it->second >= sz && (best == holes.end() || it->second < best->second)) best = it;
            if (best == holes.end()) {
                u_off[s] = top;
                top += sz;
            } else {
                u_off[s] = best->first;
                const int64_t rest = best->second - sz, off = best->first + sz;
                holes.erase(best);
                if (rest > 0) holes.emplace(off, rest);
            }
        }
    }
    stored_u = top;
    u_off[nsn] = top;
}

void symbolic_analyze(const Structure& st, Symbolic& sym) {
    const int n = st.n;
    sym = Symbolic();
    sym.n = n;
    // ---- lower pattern of K = W + J^T J + diag (original indices) ------------
    std::vector<std::pair<int32_t, int32_t>> ent;
    for (size_t e = 0; e < st.wrow.size(); ++e)
        ent.push_back({std::max(st.wrow[e], st.wcol[e]), std::min(st.wrow[e], st.wcol[e])});
    const int m = st.m_c + st.m_d;
    for (int r = 0; r < m; ++r)
        for (int p = st.jptr[r]; p < st.jptr[r + 1]; ++p)
            for (int q = st.jptr[r]; q <= p; ++q)
                ent.push_back({std::max(st.jcol[p], st.jcol[q]), std::min(st.jcol[p], st.jcol[q])});
    for (int j = 0; j < n; ++j) ent.push_back({j, j});
    std::sort(ent.begin(), ent.end());
    ent.erase(std::unique(ent.begin(), ent.end()), ent.end());
    // ---- 1. fill-reducing ordering ----------------------------------------------
    std::vector<int32_t> perm_md;
    if (st.desc.ordering == NMPC_ORDER_NESTED_DISSECTION) {
        GraphStageNd nd(n, st.H, n / st.H, st.nx, ent);
        perm_md = nd.order();
        if ((int)perm_md.size() != n) throw std::runtime_error("nested dissection: incomplete order");
    } else if (st.desc.ordering == NMPC_ORDER_FAMILY_DISSECTION && st.desc.family != NMPC_FAMILY_HEATED_PLATE) {
        perm_md = stage_nd(st.H, n / st.H);
    } else if (st.desc.ordering == NMPC_ORDER_FAMILY_DISSECTION) {
        LatticeNd nd(n, st.H, st.desc.grid, n / st.H, ent);
        perm_md = nd.order();
        if ((int)perm_md.size() != n) throw std::runtime_error("nested dissection: incomplete order");
    } else {
        Adj adj(n);
        for (auto [i, j] : ent)
            if (i != j) {
                adj[i].push_back(j);
                adj[j].push_back(i);
            }
        for (auto& a : adj) {
            std::sort(a.begin(), a.end());
            a.erase(std::unique(a.begin(), a.end()), a.end());
        }
        perm_md = min_degree(n, std::move(adj));
    }
    std::vector<int32_t> iperm(n);
    for (int k = 0; k < n; ++k) iperm[perm_md[k]] = k;
    // ---- 2-3. etree, postorder, final order -----------------------------------
    Adj strct;
    std::vector<int32_t> parent;
    column_structures(permute_lower(n, ent, iperm), strct, parent);
    std::vector<int32_t> post = postorder(parent);
    sym.perm.resize(n);
    for (int k = 0; k < n; ++k) sym.perm[k] = perm_md[post[k]];
    sym.iperm.resize(n);
    for (int k = 0; k < n; ++k) sym.iperm[sym.perm[k]] = k;
    column_structures(permute_lower(n, ent, sym.iperm), strct, parent);
    sym.parent = parent;
    sym.colcount.resize(n);
    sym.nnz_l = 0;
    sym.flops = 0;
    for (int j = 0; j < n; ++j) {
        sym.colcount[j] = (int32_t)strct[j].size();
        sym.nnz_l += sym.colcount[j];
        sym.flops += (int64_t)sym.colcount[j] * sym.colcount[j];
    }
    // ---- 4. supernodes ----------------------------------------------------------
    std::vector<int32_t> nchild(n, 0);
    for (int j = 0; j < n; ++j)
        if (parent[j] >= 0) nchild[parent[j]]++;
    std::vector<int32_t> starts{0};
    for (int j = 0; j + 1 < n; ++j) {
        bool same = parent[j] == j + 1 && nchild[j + 1] == 1 && sym.colcount[j] == sym.colcount[j + 1] + 1;
        if (!same) starts.push_back(j + 1);
    }
    std::vector<SNode> out;
    for (size_t s = 0; s < starts.size(); ++s) {
        SNode nd;
        nd.f = starts[s];
        nd.l = s + 1 < starts.size() ? starts[s + 1] : n;
        for (int32_t r : strct[nd.f])
            if (r >= nd.l) nd.below.push_back(r);
        const int64_t w = nd.l - nd.f;
        nd.stored = w * (w + 1) / 2 + w * (int64_t)nd.below.size();
        nd.zeros = 0;
        while (!out.empty()) {
            const SNode& prev = out.back();
            if (prev.l != nd.f || parent[prev.l - 1] != nd.f) break;
            const int64_t mw = nd.l - prev.f;
            const int64_t stored = mw * (mw + 1) / 2 + mw * (int64_t)nd.below.size();
            const int64_t zeros = stored - (prev.stored - prev.zeros) - (nd.stored - nd.zeros);
            const bool ok = mw <= kAmalgMaxWidth && (mw <= kAmalgSmall || 4 * zeros <= stored);
            if (!ok) break;
            nd.f = prev.f;
            nd.stored = stored;
            nd.zeros = zeros;
            out.pop_back();
        }
        out.push_back(std::move(nd));
    }
    const int nsn = (int)out.size();
    sym.nsn = nsn;
    sym.sn_ptr.resize(nsn + 1);
    sym.sn_rows_ptr.assign(nsn + 1, 0);
    for (int s = 0; s < nsn; ++s) {
        sym.sn_ptr[s] = out[s].f;
        const int w = out[s].l - out[s].f;
        sym.sn_rows_ptr[s + 1] = sym.sn_rows_ptr[s] + w + (int64_t)out[s].below.size();
    }
    sym.sn_ptr[nsn] = n;
    sym.sn_rows.resize(sym.sn_rows_ptr[nsn]);
    for (int s = 0; s < nsn; ++s) {
        int64_t o = sym.sn_rows_ptr[s];
        for (int c = out[s].f; c < out[s].l; ++c) sym.sn_rows[o++] = c;
        for (int32_t r : out[s].below) sym.sn_rows[o++] = r;
    }
    out.clear();
    std::vector<int32_t> col2sn(n);
    for (int s = 0; s < nsn; ++s)
        for (int c = sym.sn_ptr[s]; c < sym.sn_ptr[s + 1]; ++c) col2sn[c] = s;
    sym.sn_parent.assign(nsn, -1);
    for (int s = 0; s < nsn; ++s) {
        const int last = sym.sn_ptr[s + 1] - 1;
        if (parent[last] >= 0) sym.sn_parent[s] = col2sn[parent[last]];
    }
    // children lists (increasing order) and bottom-up levels
    sym.child_ptr.assign(nsn + 1, 0);
    for (int s = 0; s < nsn; ++s)
        if (sym.sn_parent[s] >= 0) sym.child_ptr[sym.sn_parent[s] + 1]++;
    for (int s = 0; s < nsn; ++s) sym.child_ptr[s + 1] += sym.child_ptr[s];
    sym.child_list.assign(sym.child_ptr[nsn], 0);
    {
        std::vector<int32_t> fill(sym.child_ptr.begin(), sym.child_ptr.end() - 1);
        for (int s = 0; s < nsn; ++s)
            if (sym.sn_parent[s] >= 0) sym.child_list[fill[sym.sn_parent[s]]++] = s;
    }
    std::vector<int32_t> lev(nsn, 0);
    int maxlev = 0;
    for (int s = 0; s < nsn; ++s) {
        for (int c = sym.child_ptr[s]; c < sym.child_ptr[s + 1]; ++c)
            lev[s] = std::max(lev[s], lev[sym.child_list[c]] + 1);
        maxlev = std::max(maxlev, lev[s]);
    }
    sym.depth = nsn ? maxlev + 1 : 0;
    sym.level_ptr.assign(sym.depth + 1, 0);
    for (int s = 0; s < nsn; ++s) sym.level_ptr[lev[s] + 1]++;
    for (int L = 0; L < sym.depth; ++L) sym.level_ptr[L + 1] += sym.level_ptr[L];
    sym.level_list.assign(nsn, 0);
    {
        std::vector<int32_t> fill(sym.level_ptr.begin(), sym.level_ptr.end() - 1);
        for (int s = 0; s < nsn; ++s) sym.level_list[fill[lev[s]]++] = s;
    }
    // storage offsets: panels and update vectors back to back; update blocks in
    // a pool where a block lives from its supernode's level until its parent's
    // level has run (best-fit reuse of released blocks)
    sym.l_off.assign(nsn + 1, 0);
    sym.u_off.assign(nsn + 1, 0);
    sym.uv_off.assign(nsn + 1, 0);
    sym.max_front = 0;
    for (int s = 0; s < nsn; ++s) {
        const int64_t w = sym.sn_ptr[s + 1] - sym.sn_ptr[s];
        const int64_t mr = sym.sn_rows_ptr[s + 1] - sym.sn_rows_ptr[s];
        sym.l_off[s + 1] = sym.l_off[s] + mr * w;
        sym.uv_off[s + 1] = sym.uv_off[s] + (mr - w);
        sym.max_front = std::max<int>(sym.max_front, (int)mr);
    }
    sym.stored_l = sym.l_off[nsn];
    sym.stored_uv = sym.uv_off[nsn];
    update_block_pool(sym, lev, sym.u_off, sym.stored_u);
    // relative positions of each supernode's below rows inside its parent's rows
    sym.rel_off.assign(nsn + 1, 0);
    for (int s = 0; s < nsn; ++s) sym.rel_off[s + 1] = sym.rel_off[s] + (sym.uv_off[s + 1] - sym.uv_off[s]);
    sym.rel.assign(sym.rel_off[nsn], 0);
    for (int s = 0; s < nsn; ++s) {
        const int p = sym.sn_parent[s];
        const int w = sym.sn_ptr[s + 1] - sym.sn_ptr[s];
        const int32_t* rs = &sym.sn_rows[sym.sn_rows_ptr[s]];
        const int64_t nb = sym.uv_off[s + 1] - sym.uv_off[s];
        if (nb == 0) continue;
        if (p < 0) throw std::runtime_error("root supernode with rows below");
        const int32_t* pb = &sym.sn_rows[sym.sn_rows_ptr[p]];
        const int32_t* pe = &sym.sn_rows[sym.sn_rows_ptr[p + 1]];
        for (int64_t t = 0; t < nb; ++t) {
            const int32_t r = rs[w + t];
            const int32_t* it = std::lower_bound(pb, pe, r);
            if (it == pe || *it != r) throw std::runtime_error("child rows not contained in parent");
            sym.rel[sym.rel_off[s] + t] = (int32_t)(it - pb);
        }
    }
    // ---- 5. KKT slots in factor order -----------------------------------------
    const int64_t nn = n;
    std::vector<int64_t> keys(ent.size());
    for (size_t e = 0; e < ent.size(); ++e) {
        int a = sym.iperm[ent[e].first], b = sym.iperm[ent[e].second];
        if (a < b) std::swap(a, b);
        keys[e] = (int64_t)b * nn + a;     // (column, row) in the permuted matrix
    }
    std::sort(keys.begin(), keys.end());
    const int64_t nk = (int64_t)keys.size();
    auto slot_of = [&](int32_t oi, int32_t oj) -> int32_t {
        int a = sym.iperm[oi], b = sym.iperm[oj];
        if (a < b) std::swap(a, b);
        const int64_t key = (int64_t)b * nn + a;
        auto it = std::lower_bound(keys.begin(), keys.end(), key);
        if (it == keys.end() || *it != key) throw std::runtime_error("KKT slot not found");
        return (int32_t)(it - keys.begin());
    };
    sym.k_fpos.resize(nk);
    sym.k_orow.resize(nk);
    sym.k_ocol.resize(nk);
    sym.k_wslot.assign(nk, -1);
    sym.k_diag.assign(nk, -1);
    sym.k_ptr.assign(nsn + 1, 0);
    sym.kcol_ptr.assign(n + 1, 0);
    for (int64_t t = 0; t < nk; ++t) {
        const int32_t pj = (int32_t)(keys[t] / nn), pi = (int32_t)(keys[t] % nn);
        const int s = col2sn[pj];
        const int32_t* rb = &sym.sn_rows[sym.sn_rows_ptr[s]];
        const int32_t* re = &sym.sn_rows[sym.sn_rows_ptr[s + 1]];
        const int32_t* it = std::lower_bound(rb, re, pi);
        if (it == re || *it != pi) throw std::runtime_error("KKT entry outside the factor pattern");
        const int64_t ld = (re - rb) | 1;   // fronts use an odd leading dimension
        sym.k_fpos[t] = (int32_t)((it - rb) + (int64_t)(pj - sym.sn_ptr[s]) * ld);
        const int32_t oi = sym.perm[pi], oj = sym.perm[pj];
        sym.k_orow[t] = std::max(oi, oj);
        sym.k_ocol[t] = std::min(oi, oj);
        if (pi == pj) sym.k_diag[t] = oi;
        sym.k_ptr[s + 1]++;
        sym.kcol_ptr[pj + 1]++;
    }
    for (int s = 0; s < nsn; ++s) sym.k_ptr[s + 1] += sym.k_ptr[s];
    for (int j = 0; j < n; ++j) sym.kcol_ptr[j + 1] += sym.kcol_ptr[j];
    for (size_t e = 0; e < st.wrow.size(); ++e) {
        const int32_t t = slot_of(st.wrow[e], st.wcol[e]);
        if (sym.k_wslot[t] >= 0) throw std::runtime_error("duplicate Hessian slot");
        sym.k_wslot[t] = (int32_t)e;
    }
    // J^T Q J contributions: every pair of entries of every constraint row
    struct Contrib { int32_t slot, a, b, r; };
    std::vector<Contrib> cs;
    for (int r = 0; r < m; ++r)
        for (int p = st.jptr[r]; p < st.jptr[r + 1]; ++p)
            for (int q = st.jptr[r]; q <= p; ++q) cs.push_back({slot_of(st.jcol[p], st.jcol[q]), p, q, r});
    std::stable_sort(cs.begin(), cs.end(), [](const Contrib& x, const Contrib& y) { return x.slot < y.slot; });
    sym.kc_ptr.assign(nk + 1, 0);
    sym.kc_a.resize(cs.size());
    sym.kc_b.resize(cs.size());
    sym.kc_r.resize(cs.size());
    for (size_t e = 0; e < cs.size(); ++e) {
        sym.kc_ptr[cs[e].slot + 1]++;
        sym.kc_a[e] = cs[e].a;
        sym.kc_b[e] = cs[e].b;
        sym.kc_r[e] = cs[e].r;
    }
    for (int64_t t = 0; t < nk; ++t) sym.kc_ptr[t + 1] += sym.kc_ptr[t];
    // transposed Jacobian (per variable: slots and rows, rows ascending)
    sym.jt_ptr.assign(n + 1, 0);
    for (size_t p = 0; p < st.jcol.size(); ++p) sym.jt_ptr[st.jcol[p] + 1]++;
    for (int j = 0; j < n; ++j) sym.jt_ptr[j + 1] += sym.jt_ptr[j];
    sym.jt_slot.resize(st.jcol.size());
    sym.jt_row.resize(st.jcol.size());
    {
        std::vector<int32_t> fill(sym.jt_ptr.begin(), sym.jt_ptr.end() - 1);
        for (int r = 0; r < m; ++r)
            for (int p = st.jptr[r]; p < st.jptr[r + 1]; ++p) {
                const int32_t j = st.jcol[p];
                sym.jt_slot[fill[j]] = p;
                sym.jt_row[fill[j]] = r;
                fill[j]++;
            }
    }
}

}  // namespace nmpc
