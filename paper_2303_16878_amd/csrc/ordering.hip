// Host-side orderings of the 6 NP x 6 NP pose system for the blocked Cholesky factorisation.
//
// The system couples two pose variables exactly when some pair links them (Sec. IV, the
// pairwise photometric terms), so its block pattern is the pose graph's adjacency.  In the
// natural order a trajectory with loop closures factors as one long chain of dependent block
// columns.  A nested-dissection order (recursive graph bisection by a vertex separator,
// separators numbered last) turns the elimination tree of 64-wide block columns into a shallow
// tree: columns of one tree level are independent and factor together.
//
// Each dissection block (a leaf or a separator) starts on a 64-row boundary of the factored
// system, padded with rows that have a unit diagonal and no coupling, so that no block column
// mixes variables of independent subtrees.

#include "pba_internal.h"

#include <algorithm>
#include <map>

namespace pba {

namespace {

// Breadth-first levels from `start` over the vertices with in[v] set; dist[v] = -1 elsewhere.
// Returns the vertices reached, in visiting order.
std::vector<int> bfs_levels(const std::vector<std::vector<int>> &adj, const std::vector<char> &in, int start,
                            std::vector<int> &dist)
{
    std::vector<int> seen{start};
    dist[start] = 0;
    for (size_t h = 0; h < seen.size(); ++h) {
        const int u = seen[h];
        for (int v : adj[u])
            if (in[v] && dist[v] < 0) {
                dist[v] = dist[u] + 1;
                seen.push_back(v);
            }
    }
    return seen;
}

struct Dissector {
    const std::vector<std::vector<int>> &adj;
    int leaf;
    std::vector<char> in;
    std::vector<int> dist;
    std::vector<std::vector<int>> blocks;   // output: leaves and separators, children first

    void emit(std::vector<int> nodes)
    {
        std::sort(nodes.begin(), nodes.end());
        blocks.push_back(std::move(nodes));
    }

    // Breadth-first levels from `start` within the vertices marked in in[]; the vertices reached.
    std::vector<int> levels_from(int start)
    {
        return bfs_levels(adj, in, start, dist);
    }

    void clear(const std::vector<int> &nodes)
    {
        for (int v : nodes) dist[v] = -1;
    }

    void split(std::vector<int> nodes)
    {
        if ((int)nodes.size() <= leaf) {
            emit(std::move(nodes));
            return;
        }
        for (int v : nodes) in[v] = 1;
        // a pseudo-peripheral start: two sweeps, each restarting from the smallest-numbered
        // vertex of the deepest level
        int s = *std::min_element(nodes.begin(), nodes.end());
        for (int sweep = 0; sweep < 2; ++sweep) {
            const std::vector<int> seen = levels_from(s);
            int best = s;
            for (int v : seen)
                if (dist[v] > dist[best] || (dist[v] == dist[best] && v < best)) best = v;
            clear(seen);
            s = best;
        }
        const std::vector<int> seen = levels_from(s);
        std::vector<int> lev(nodes.size());
        for (size_t i = 0; i < nodes.size(); ++i) lev[i] = dist[nodes[i]];
        clear(seen);
        for (int v : nodes) in[v] = 0;
        if (seen.size() < nodes.size()) {   // disconnected: the reached component, then the rest
            std::vector<int> a, b;
            for (size_t i = 0; i < nodes.size(); ++i) (lev[i] >= 0 ? a : b).push_back(nodes[i]);
            split(std::move(a));
            split(std::move(b));
            return;
        }
        // the level of the median vertex (ordered by level, then number) is the separator
        std::vector<std::pair<int, int>> order(nodes.size());
        for (size_t i = 0; i < nodes.size(); ++i) order[i] = {lev[i], nodes[i]};
        std::sort(order.begin(), order.end());
        const int mid = order[order.size() / 2].first;
        std::vector<int> left, right, sep;
        for (size_t i = 0; i < nodes.size(); ++i)
            (lev[i] < mid ? left : lev[i] > mid ? right : sep).push_back(nodes[i]);
        if (left.empty() || right.empty()) {
            emit(std::move(nodes));
            return;
        }
        split(std::move(left));
        split(std::move(right));
        emit(std::move(sep));
    }
};

}  // namespace

std::vector<std::vector<int>> nd_blocks(int nv, const std::vector<std::pair<int, int>> &edges, int leaf)
{
    std::vector<std::vector<int>> adj(nv);
    for (const auto &e : edges)
        if (e.first != e.second) {
            adj[e.first].push_back(e.second);
            adj[e.second].push_back(e.first);
        }
    for (auto &a : adj) {
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
    }
    Dissector d{adj, std::max(1, leaf), std::vector<char>(nv, 0), std::vector<int>(nv, -1), {}};
    std::vector<int> all(nv);
    for (int v = 0; v < nv; ++v) all[v] = v;
    if (nv > 0) d.split(std::move(all));
    return std::move(d.blocks);
}

TilePattern tile_pattern(int n, const std::vector<int> &pos, const std::vector<std::pair<int, int>> &edges)
{
    TilePattern tp;
    tp.n = n;
    const int nt = tp.nt = (n + 63) / 64;
    std::vector<char> occ((size_t)nt * nt, 0);   // lower triangle: occ[i * nt + j], i >= j
    auto mark = [&](int a, int b) {
        const int ta[2] = {pos[a] / 64, (pos[a] + 5) / 64}, tb[2] = {pos[b] / 64, (pos[b] + 5) / 64};
        for (int x : ta)
            for (int y : tb) occ[(size_t)std::max(x, y) * nt + std::min(x, y)] = 1;
    };
    for (int v = 0; v < (int)pos.size(); ++v) mark(v, v);
    for (const auto &e : edges) mark(e.first, e.second);
    for (int k = 0; k < nt; ++k) occ[(size_t)k * nt + k] = 1;
    tp.rows.assign(nt, {});
    for (int k = 0; k < nt; ++k) {
        std::vector<int> &r = tp.rows[k];
        for (int i = k + 1; i < nt; ++i)
            if (occ[(size_t)i * nt + k]) r.push_back(i);
        // symbolic fill of this column's update
        for (size_t a = 0; a < r.size(); ++a)
            for (size_t b = 0; b <= a; ++b) occ[(size_t)r[a] * nt + r[b]] = 1;
    }
    tp.cols.assign(nt, {});
    for (int k = 0; k < nt; ++k)
        for (int j = 0; j < k; ++j)
            if (occ[(size_t)k * nt + j]) tp.cols[k].push_back(j);
    // elimination tree of the block columns (parent = first tile row below the diagonal) and each
    // column's height above the leaves: the tiles a column's update writes all belong to its
    // ancestors, which are on strictly higher levels
    tp.level.assign(nt, 0);
    for (int k = 0; k < nt; ++k)
        if (!tp.rows[k].empty()) {
            const int p = tp.rows[k][0];
            tp.level[p] = std::max(tp.level[p], tp.level[k] + 1);
        }
    tp.nlev = nt ? *std::max_element(tp.level.begin(), tp.level.end()) + 1 : 0;
    return tp;
}

std::vector<int> nd_positions(int nv, const std::vector<std::vector<int>> &blocks, int &n_pad)
{
    std::vector<int> pos(nv, -1);
    int off = 0;
    for (const auto &b : blocks) {
        for (size_t j = 0; j < b.size(); ++j) pos[b[j]] = off + 6 * (int)j;
        off += (6 * (int)b.size() + 63) / 64 * 64;
    }
    n_pad = off;
    return pos;
}

NdArrays nd_arrays(const TilePattern &tp, const std::vector<int> &pos)
{
    NdArrays a;
    const int nt = tp.nt;
    a.perm.assign(tp.n, -1);
    for (int v = 0; v < (int)pos.size(); ++v)
        for (int i = 0; i < 6; ++i) a.perm[pos[v] + i] = 6 * v + i;
    for (int k = 0; k < nt; ++k) {   // every lower tile of the pattern, column by column
        a.dtiles.insert(a.dtiles.end(), {k, k});
        for (int i : tp.rows[k]) a.dtiles.insert(a.dtiles.end(), {i, k});
    }
    for (int l = 0; l < tp.nlev; ++l) {
        a.lbeg.push_back((int)a.lcols.size());
        // target tile (a, b), b <= a -> the level's columns having both among their tile rows
        std::map<std::pair<int, int>, std::vector<int32_t>> tgt_of;
        for (int k = 0; k < nt; ++k) {
            if (tp.level[k] != l) continue;
            a.lcols.push_back(k);
            const std::vector<int> &r = tp.rows[k];
            for (size_t x = 0; x < r.size(); ++x)
                for (size_t y = 0; y <= x; ++y) tgt_of[{r[x], r[y]}].push_back(k);
        }
        a.lcnt.push_back((int)a.lcols.size() - a.lbeg.back());
        // the tasks with the most contributors first, so that they start early
        std::vector<std::pair<std::pair<int, int>, const std::vector<int32_t> *>> tl;
        for (const auto &t : tgt_of) tl.push_back({t.first, &t.second});
        std::stable_sort(tl.begin(), tl.end(),
                         [](const auto &x, const auto &y) { return x.second->size() > y.second->size(); });
        a.tbeg.push_back((int)a.tasks.size() / 4);
        for (const auto &t : tl) {
            a.tasks.insert(a.tasks.end(), {t.first.first, t.first.second, (int32_t)a.contrib.size(),
                                           (int32_t)t.second->size()});
            a.contrib.insert(a.contrib.end(), t.second->begin(), t.second->end());
        }
        a.tcnt.push_back((int)a.tasks.size() / 4 - a.tbeg.back());
    }
    return a;
}

}  // namespace pba
