// Host-side bandwidth-reducing renumbering (reverse Cuthill-McKee) of a
// sparse matrix whose numbering scatters the columns of neighbouring rows,
// and the measure that decides whether it is worth applying.
//
// The fused step gathers x through the column indices of each 64-row slice;
// when the rows of a slice couple to columns far apart, every lane's gather
// touches its own cache line.  Cuthill-McKee numbers the graph of the matrix
// by breadth-first levels from a peripheral vertex, neighbours in increasing
// degree, so the rows of a slice couple to a few short column ranges in the
// neighbouring levels; reversing the order keeps that and reduces fill
// profile (the textbook reverse form).
#pragma once
#include <algorithm>
#include <cstdint>
#include <numeric>
#include <vector>

namespace pprc {

// Mean number of distinct 64-byte lines (8 doubles) of x that one slice of 64
// consecutive rows gathers, per stored entry, over `samples` slices spread over
// the matrix (1 = every entry its own line, 1/8 = perfectly contiguous).
// perm (new -> old) and iperm (old -> new) renumber the matrix, or are empty.
inline double gather_spread(int64_t n, const std::vector<int64_t> &rp, const std::vector<int32_t> &col,
                            const std::vector<int64_t> &perm, const std::vector<int64_t> &iperm, int samples = 2048)
{
    const int64_t ns = (n + 63) / 64;
    const int64_t step = std::max<int64_t>(1, ns / samples);
    int64_t lines = 0, entries = 0;
    std::vector<int64_t> ln;
    for (int64_t s = 0; s < ns; s += step) {
        ln.clear();
        for (int64_t r = s * 64; r < std::min(n, s * 64 + 64); ++r) {
            const int64_t o = perm.empty() ? r : perm[r];
            for (int64_t p = rp[o]; p < rp[o + 1]; ++p) {
                const int64_t c = iperm.empty() ? col[p] : iperm[col[p]];
                ln.push_back(c >> 3);
            }
        }
        entries += (int64_t)ln.size();
        std::sort(ln.begin(), ln.end());
        lines += (int64_t)(std::unique(ln.begin(), ln.end()) - ln.begin());
    }
    return entries > 0 ? (double)lines / (double)entries : 0.0;
}

// Breadth-first levels from `root` over unvisited vertices; returns the last
// vertex reached of smallest degree and the number of levels.
inline int64_t bfs_far(int64_t root, const std::vector<int64_t> &rp, const std::vector<int32_t> &col,
                       const std::vector<int64_t> &deg, std::vector<int32_t> &mark, int32_t stamp, int *levels)
{
    std::vector<int64_t> cur{root}, nxt;
    mark[root] = stamp;
    int lv = 1;
    int64_t best = root;
    while (true) {
        nxt.clear();
        for (int64_t u : cur)
            for (int64_t p = rp[u]; p < rp[u + 1]; ++p) {
                const int64_t v = col[p];
                if (mark[v] != stamp && mark[v] >= 0) {
                    mark[v] = stamp;
                    nxt.push_back(v);
                }
            }
        if (nxt.empty()) break;
        ++lv;
        cur.swap(nxt);
    }
    best = cur[0];
    for (int64_t v : cur)
        if (deg[v] < deg[best]) best = v;
    *levels = lv;
    return best;
}

// Reverse Cuthill-McKee: perm[new] = old.  Components are numbered one after
// the other, each from a pseudo-peripheral vertex (repeated breadth-first
// searches from the far end while the level count grows).
inline std::vector<int64_t> rcm(int64_t n, const std::vector<int64_t> &rp, const std::vector<int32_t> &col)
{
    std::vector<int64_t> deg(n);
    for (int64_t i = 0; i < n; ++i) deg[i] = rp[i + 1] - rp[i];
    std::vector<int32_t> mark(n, 0);   // > 0: search stamps; -1: numbered
    std::vector<int64_t> order;
    order.reserve(n);
    std::vector<int64_t> by_deg(n);
    std::iota(by_deg.begin(), by_deg.end(), 0);
    std::stable_sort(by_deg.begin(), by_deg.end(), [&](int64_t a, int64_t b) { return deg[a] < deg[b]; });
    int32_t stamp = 0;
    std::vector<int64_t> nb;
    for (int64_t start : by_deg) {
        if (mark[start] < 0) continue;
        int lv = 0, lv_prev = -1;
        int64_t root = start;
        for (int t = 0; t < 4; ++t) {
            const int64_t far = bfs_far(root, rp, col, deg, mark, ++stamp, &lv);
            if (lv <= lv_prev) break;
            lv_prev = lv;
            root = far;
        }
        // Cuthill-McKee from root
        const size_t head0 = order.size();
        order.push_back(root);
        mark[root] = -1;
        for (size_t h = head0; h < order.size(); ++h) {
            const int64_t u = order[h];
            nb.clear();
            for (int64_t p = rp[u]; p < rp[u + 1]; ++p) {
                const int64_t v = col[p];
                if (mark[v] >= 0) {
                    mark[v] = -1;
                    nb.push_back(v);
                }
            }
            std::sort(nb.begin(), nb.end(), [&](int64_t a, int64_t b) {
                return deg[a] != deg[b] ? deg[a] < deg[b] : a < b;
            });
            order.insert(order.end(), nb.begin(), nb.end());
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

}  // namespace pprc
