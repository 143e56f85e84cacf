// Clustered block partition (Section 6.1 and eq. (extended_set) of Section
// 6.1.1: the blocks should keep their neighbourhoods N_j small; the paper
// partitions the free-set graph with an external graph partitioner). Host
// code: blocks grown breadth-first on the graph of the free pairs.
//
//   * vertices 0..n-1, an edge for every free pair (i, j), i != j;
//   * blocks of exactly b vertices (the last one shorter), formed one after
//     another; the variables are relabelled in block order, so that the
//     solver's contiguous blocks are the clusters;
//   * a block grows breadth-first from a seed over vertices not yet placed
//     (neighbours visited in ascending order) until it holds b vertices; when
//     its component is exhausted it continues from the next seed;
//   * the next seed is the oldest unplaced vertex among the candidates (the
//     vertices adjacent to an earlier block, queued when that block was
//     completed: block members in order, each one's neighbours ascending),
//     else the unplaced vertex of least degree (ties: smaller index).
// O(n + pairs) time and memory.
#include <algorithm>
#include <deque>
#include <numeric>

#include "sic_steps.h"
#include "solver.h"

namespace sic {

std::vector<int32_t> cluster_order(int64_t n, const int64_t* keys, int64_t count, int b) {
    if (n < 1 || b < 1) throw SicError(SIC_EINVAL, "cluster_order: bad sizes");
    // neighbour lists as a CSR (both directions, sorted, duplicates removed)
    std::vector<int64_t> ptr(n + 1, 0);
    for (int64_t t = 0; t < count; ++t) {
        const int64_t i = keys[t] / n, j = keys[t] % n;
        if (i < 0 || i >= n || j < 0 || j >= n) throw SicError(SIC_EINVAL, "cluster_order: key out of range");
        if (i == j) continue;
        ++ptr[i + 1];
        ++ptr[j + 1];
    }
    for (int64_t v = 0; v < n; ++v) ptr[v + 1] += ptr[v];
    std::vector<int32_t> nb(ptr[n]);
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t t = 0; t < count; ++t) {
        const int64_t i = keys[t] / n, j = keys[t] % n;
        if (i == j) continue;
        nb[fill[i]++] = (int32_t)j;
        nb[fill[j]++] = (int32_t)i;
    }
    std::vector<int64_t> deg(n);
    for (int64_t v = 0; v < n; ++v) {
        auto b0 = nb.begin() + ptr[v], b1 = nb.begin() + ptr[v + 1];
        std::sort(b0, b1);
        deg[v] = std::unique(b0, b1) - b0;
    }
    std::vector<int32_t> by_degree(n);
    std::iota(by_degree.begin(), by_degree.end(), 0);
    std::stable_sort(by_degree.begin(), by_degree.end(),
                     [&](int32_t a, int32_t c) { return deg[a] < deg[c]; });
    std::vector<char> placed(n, 0);
    std::deque<int32_t> cand, queue;
    std::vector<int32_t> order;
    order.reserve(n);
    std::vector<int32_t> block;
    size_t sp = 0;
    while ((int64_t)order.size() < n) {
        const int64_t need = std::min<int64_t>(b, n - (int64_t)order.size());
        block.clear();
        while ((int64_t)block.size() < need) {
            int32_t seed = -1;
            while (!cand.empty()) {
                const int32_t v = cand.front();
                cand.pop_front();
                if (!placed[v]) {
                    seed = v;
                    break;
                }
            }
            if (seed < 0) {
                while (placed[by_degree[sp]]) ++sp;
                seed = by_degree[sp];
            }
            placed[seed] = 1;
            block.push_back(seed);
            queue.clear();
            queue.push_back(seed);
            while (!queue.empty() && (int64_t)block.size() < need) {
                const int32_t u = queue.front();
                queue.pop_front();
                for (int64_t e = ptr[u]; e < ptr[u] + deg[u]; ++e) {
                    if ((int64_t)block.size() == need) break;
                    const int32_t w = nb[e];
                    if (!placed[w]) {
                        placed[w] = 1;
                        block.push_back(w);
                        queue.push_back(w);
                    }
                }
            }
        }
        for (int32_t u : block)
            for (int64_t e = ptr[u]; e < ptr[u] + deg[u]; ++e)
                if (!placed[nb[e]]) cand.push_back(nb[e]);
        order.insert(order.end(), block.begin(), block.end());
    }
    return order;
}

}  // namespace sic

extern "C" int sic_cluster_order(int64_t n, const int64_t* keys, int64_t count, int b,
                                 int32_t* order_out) {
    if (n < 1 || n > INT32_MAX || b < 1 || count < 0 || (count > 0 && !keys) || !order_out)
        return SIC_EINVAL;
    try {
        const std::vector<int32_t> o = sic::cluster_order(n, keys, count, b);
        std::copy(o.begin(), o.end(), order_out);
        return SIC_OK;
    } catch (const sic::SicError& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        return SIC_ENOMEM;
    }
}
