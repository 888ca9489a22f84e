// PC steps 2 and 3 (Section III-C): orientation of a learned skeleton into a
// CPDAG, on the host (a few operations per edge; the skeleton search is the
// hot path).
//
// Step 2 orients x -> z <- y for every unshielded triple x - z - y whose
// middle node z is not in SepSet(x, y); all triples are judged on the
// skeleton, and an edge two triples orient both ways keeps both arrowheads.
// Step 3 applies Meek's rules R1-R3 to the undirected edges, with only
// singly-directed edges as premises, in rounds: every orientation a round
// implies is collected on the graph as it stood, then all are applied; an
// edge one round orients both ways keeps both arrowheads.
#include <algorithm>
#include <cstring>
#include <utility>
#include <vector>

#include "skeleton.h"

namespace {

struct Marks {
    int n;
    std::vector<int8_t> m;  // m[i * n + j]: 0 not adjacent, 1 no arrowhead at j, 2 arrowhead at j
    int8_t at(int i, int j) const { return m[(size_t)i * n + j]; }
    bool adjacent(int i, int j) const { return at(i, j) != 0; }
    bool directed(int i, int j) const { return at(i, j) == 2 && at(j, i) == 1; }
    bool undirected(int i, int j) const { return at(i, j) == 1 && at(j, i) == 1; }
};

bool in_sepset(const bns_skeleton &sk, int x, int y, int z) {
    const int64_t ij = (int64_t)x * sk.n + y;
    const int32_t d = sk.depth[ij];
    if (d <= 0) return false;  // removed with the empty set (depth 0)
    const int32_t *s = sk.pool.data() + sk.sepoff[ij];
    return std::binary_search(s, s + d, z);  // members are ascending
}

}  // namespace

extern "C" bns_status bns_skeleton_orient(const bns_skeleton *sk, int8_t *cpdag) {
    if (!sk || !cpdag) return BNS_E_INVALID_ARG;
    sk->expand();
    const int n = sk->n;
    Marks G{n, std::vector<int8_t>((size_t)n * n, 0)};
    // neighbour lists (ascending) of the skeleton
    std::vector<std::vector<int>> nb((size_t)n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (i != j && sk->adj[(size_t)i * n + j]) {
                nb[i].push_back(j);
                G.m[(size_t)i * n + j] = 1;
            }
    // step 2: unshielded colliders
    std::vector<uint8_t> head((size_t)n * n, 0);
    for (int z = 0; z < n; ++z) {
        const std::vector<int> &a = nb[z];
        for (size_t p = 0; p < a.size(); ++p)
            for (size_t q = p + 1; q < a.size(); ++q) {
                const int x = a[p], y = a[q];  // x < y
                if (sk->adj[(size_t)x * n + y]) continue;
                if (in_sepset(*sk, x, y, z)) continue;
                head[(size_t)x * n + z] = head[(size_t)y * n + z] = 1;
            }
    }
    for (size_t k = 0; k < head.size(); ++k)
        if (head[k]) G.m[k] = 2;
    // step 3: Meek rounds
    std::vector<std::pair<int, int>> found;
    std::vector<uint8_t> mark((size_t)n * n, 0);  // orientations found this round
    std::vector<int> cs;
    for (;;) {
        found.clear();
        for (int a = 0; a < n; ++a)
            for (int b : nb[a]) {
                if (!G.undirected(a, b)) continue;
                bool hit = false;
                // R1: c -> a, c and b not adjacent
                for (int c : nb[a])
                    if (c != b && G.directed(c, a) && !G.adjacent(c, b)) {
                        hit = true;
                        break;
                    }
                // R2: a -> c -> b
                if (!hit)
                    for (int c : nb[a])
                        if (c != b && G.directed(a, c) && G.directed(c, b)) {
                            hit = true;
                            break;
                        }
                // R3: a - c -> b and a - d -> b, c and d not adjacent
                if (!hit) {
                    cs.clear();
                    for (int c : nb[a])
                        if (c != b && G.undirected(a, c) && G.directed(c, b)) cs.push_back(c);
                    for (size_t p = 0; p < cs.size() && !hit; ++p)
                        for (size_t q = p + 1; q < cs.size(); ++q)
                            if (!G.adjacent(cs[p], cs[q])) {
                                hit = true;
                                break;
                            }
                }
                if (hit) found.emplace_back(a, b);
            }
        if (found.empty()) break;
        for (const auto &f : found) mark[(size_t)f.first * n + f.second] = 1;
        for (const auto &f : found) {
            const int a = f.first, b = f.second;
            G.m[(size_t)a * n + b] = 2;
            if (!mark[(size_t)b * n + a]) G.m[(size_t)b * n + a] = 1;
        }
        for (const auto &f : found) mark[(size_t)f.first * n + f.second] = 0;
    }
    std::memcpy(cpdag, G.m.data(), G.m.size());
    return BNS_OK;
}

extern "C" bns_status bns_skeleton_create(int32_t n, const uint8_t *adj, const int32_t *depth,
                                          const int64_t *sep_off, const int32_t *pool, int64_t pool_len,
                                          bns_skeleton **out) {
    if (!out) return BNS_E_INVALID_ARG;
    *out = nullptr;
    if (n < 2 || n > 65535 || !adj || !depth || !sep_off || pool_len < 0 || (pool_len > 0 && !pool))
        return BNS_E_INVALID_ARG;
    bns_skeleton *sk = new bns_skeleton();
    sk->full = true;
    sk->n = n;
    const size_t nn = (size_t)n * n;
    sk->adj.assign(adj, adj + nn);
    sk->depth.assign(depth, depth + nn);
    sk->sepoff.assign(sep_off, sep_off + nn);
    sk->pool.assign(pool, pool + pool_len);
    bool ok = true;
    for (int i = 0; i < n && ok; ++i)
        for (int j = 0; j < n && ok; ++j) {
            const size_t ij = (size_t)i * n + j, ji = (size_t)j * n + i;
            if (i == j) {
                ok = adj[ij] == 0;
                continue;
            }
            const int32_t d = depth[ij];
            ok = adj[ij] == adj[ji] && depth[ij] == depth[ji] && adj[ij] <= 1 && (adj[ij] ? d == -1 : d >= 0);
            if (!ok || adj[ij]) continue;
            if (d == 0) continue;
            const int64_t o = sep_off[ij];
            ok = o >= 0 && o + d <= pool_len;
            for (int32_t k = 0; ok && k < d; ++k) {
                const int32_t v = pool[o + k];
                ok = v >= 0 && v < n && v != i && v != j && (k == 0 || pool[o + k - 1] < v);
            }
        }
    if (!ok) {
        delete sk;
        return BNS_E_INVALID_ARG;
    }
    *out = sk;
    return BNS_OK;
}
