// Host construction of a mesh's tiled layout (plain C++, no device code):
// node numbering, tet order, tiles, the dealing of each tile's tets to
// wavefront lanes, and the node -> tile entry lists. The library builds it
// once per mesh; a CPU test program builds it under the address and
// undefined-behaviour sanitizers.
#pragma once

#include <algorithm>
#include <bitset>
#include <cstdint>
#include <utility>
#include <vector>

namespace fem_layout {

// ---------------------------------------------------------------------------
// Tiled layout of one mesh (host construction).
// ---------------------------------------------------------------------------
struct HostLayout {
    int n = 0, m = 0, ntile = 0, nent = 0;
    std::vector<int> tile_tet, tile_ent, ent_node, node_ent_off, node_ent;
    std::vector<uint32_t> tet_loc;
    std::vector<int> order;             // tile position -> input tet index
    std::vector<int> tet_nodes;         // 4 x m: global node ids per tet in tile order and device vertex order
};

inline uint32_t spread_bits(uint32_t v) {   // 10 bits -> every third bit
    v &= 0x3ff;
    v = (v | (v << 16)) & 0x030000ff;
    v = (v | (v << 8)) & 0x0300f00f;
    v = (v | (v << 4)) & 0x030c30c3;
    v = (v | (v << 2)) & 0x09249249;
    return v;
}

// Tets in Morton order of their centroids, cut greedily into tiles of at most
// kTileTets tets and kTileNodes distinct nodes.
// Order and vertex rotation of a tile's tets for the device. The tile
// kernels hand 64 consecutive tets to one wavefront, which accumulates into
// LDS one local node slot at a time with 64-bit atomics; lanes that share a
// node in one slot serialise on one address, and the LDS serves such an
// instruction 16 lanes at a time, where nodes whose local ids agree mod 16
// fall on one bank. Tets are dealt greedily to quarters of 16 positions (the
// last one holds the remainder), each also free to take one of the 12 even
// vertex orders (orientation, hence the sign of det D_m, is kept): first
// avoiding a node repeated in one slot within a group of 64, then a bank
// repeated in one slot within a quarter; ties go to the emptiest quarter.
// placed[j] = (index into words) * 16 + order, for position j.
inline constexpr int kEvenPerm[12][4] = {{0, 1, 2, 3}, {0, 2, 3, 1}, {0, 3, 1, 2}, {1, 0, 3, 2}, {1, 2, 0, 3}, {1, 3, 2, 0},
                                  {2, 0, 1, 3}, {2, 1, 3, 0}, {2, 3, 0, 1}, {3, 0, 2, 1}, {3, 1, 0, 2}, {3, 2, 1, 0}};

inline void spread_tile(const std::vector<uint32_t> &words, std::vector<int> &placed) {
    const int nk = (int)words.size();
    const int ng = (nk + 63) / 64;
    const int nq = (nk + 15) / 16;
    std::vector<int> cap(nq, 16);
    if (nq > 0) cap[nq - 1] = nk - 16 * (nq - 1);
    std::vector<std::bitset<256>> used((size_t)ng * 4);   // nodes per group and slot
    std::vector<uint32_t> bank((size_t)nq * 4, 0u);       // local id mod 16 per quarter and slot
    std::vector<std::vector<int>> members(nq);
    for (int t = 0; t < nk; t++) {
        int l[4];
        for (int a = 0; a < 4; a++) l[a] = (words[t] >> (8 * a)) & 0xff;
        int best = -1, best_perm = 0, best_cost = 1 << 30, best_room = -1;
        for (int q = 0; q < nq; q++) {
            const int room = cap[q] - (int)members[q].size();
            if (room == 0) continue;
            const int g = q / 4;
            for (int r = 0; r < 12; r++) {
                int cost = 0;
                for (int a = 0; a < 4; a++) {
                    const int v = l[kEvenPerm[r][a]];
                    cost += used[4 * g + a][v] ? 64 : 0;
                    cost += (bank[4 * q + a] >> (v & 15)) & 1u;
                }
                if (cost < best_cost || (cost == best_cost && room > best_room)) {
                    best = q;
                    best_perm = r;
                    best_cost = cost;
                    best_room = room;
                }
            }
        }
        members[best].push_back(t * 16 + best_perm);
        for (int a = 0; a < 4; a++) {
            const int v = l[kEvenPerm[best_perm][a]];
            used[4 * (best / 4) + a].set(v);
            bank[4 * best + a] |= 1u << (v & 15);
        }
    }
    placed.clear();
    for (const std::vector<int> &q : members) placed.insert(placed.end(), q.begin(), q.end());
}

// Tets sorted along a Morton curve of their centroids (10 bits per axis over
// the mesh's bounding cube); ties keep input order.
inline std::vector<int> morton_order(const double *X, int n, const int32_t *tets, int m) {
    double lo[3] = {X[0], X[1], X[2]}, hi[3] = {X[0], X[1], X[2]};
    for (int i = 0; i < n; i++)
        for (int d = 0; d < 3; d++) {
            lo[d] = std::min(lo[d], X[3 * i + d]);
            hi[d] = std::max(hi[d], X[3 * i + d]);
        }
    double ext = 0.0;
    for (int d = 0; d < 3; d++) ext = std::max(ext, hi[d] - lo[d]);
    if (!(ext > 0.0)) ext = 1.0;
    std::vector<std::pair<uint32_t, int>> key(m);
    for (int e = 0; e < m; e++) {
        uint32_t code = 0;
        for (int d = 0; d < 3; d++) {
            double c = 0.0;
            for (int a = 0; a < 4; a++) c += X[3 * tets[4 * e + a] + d];
            c = 0.25 * c;
            int q = (int)((c - lo[d]) / ext * 1023.0);
            q = std::max(0, std::min(1023, q));
            code |= spread_bits((uint32_t)q) << d;
        }
        key[e] = {code, e};
    }
    std::sort(key.begin(), key.end());
    std::vector<int> order(m);
    for (int k = 0; k < m; k++) order[k] = key[k].second;
    return order;
}

// Device node numbering: nodes numbered by first touch along the tets'
// Morton order, so the nodes a tile touches are mostly consecutive and its
// gathers of node vectors read whole cache lines. perm[new] = input id.
inline std::vector<int> node_order(const double *X, int n, const int32_t *tets, int m) {
    const std::vector<int> order = morton_order(X, n, tets, m);
    std::vector<int> perm;
    std::vector<char> seen(n, 0);
    perm.reserve(n);
    for (int e : order)
        for (int a = 0; a < 4; a++) {
            const int v = tets[4 * e + a];
            if (!seen[v]) {
                seen[v] = 1;
                perm.push_back(v);
            }
        }
    for (int v = 0; v < n; v++)
        if (!seen[v]) perm.push_back(v);
    return perm;
}

inline void build_layout(const double *X, int n, const int32_t *tets, int m, int max_tets, int max_nodes, HostLayout &L) {
    L.n = n;
    L.m = m;
    const std::vector<int> order = morton_order(X, n, tets, m);
    std::vector<int> stamp(n, -1), local(n, 0);
    L.tile_tet.assign(1, 0);
    L.tile_ent.assign(1, 0);
    L.ent_node.clear();
    L.tet_loc.assign(m, 0);
    L.order.assign(m, 0);
    L.tet_nodes.assign(4 * (size_t)m, 0);
    int tile = 0, tile_tets = 0, tile_nodes = 0, pos = 0;
    std::vector<int> tile_list;
    std::vector<uint32_t> words;
    std::vector<int> elems, placed;
    auto close_tile = [&]() {
        std::sort(tile_list.begin(), tile_list.end());   // entries in ascending node order
        for (size_t k = 0; k < tile_list.size(); k++) local[tile_list[k]] = (int)k;
        const int t0 = L.tile_tet.back();
        words.clear();
        elems.clear();
        for (int k = t0; k < pos; k++) {
            const int e = order[k];
            uint32_t w = 0;
            for (int a = 0; a < 4; a++) w |= (uint32_t)local[tets[4 * e + a]] << (8 * a);
            words.push_back(w);
            elems.push_back(e);
        }
        spread_tile(words, placed);
        for (int k = t0; k < pos; k++) {
            const int src = placed[k - t0] >> 4, r = placed[k - t0] & 15;
            const int e = elems[src];
            uint32_t w = 0;
            for (int a = 0; a < 4; a++) {
                const int from = kEvenPerm[r][a];
                w |= ((words[src] >> (8 * from)) & 0xffu) << (8 * a);
                L.tet_nodes[4 * (size_t)k + a] = tets[4 * (size_t)e + from];
            }
            L.tet_loc[k] = w;
            L.order[k] = e;
        }
        for (int v : tile_list) L.ent_node.push_back(v);
        L.tile_tet.push_back(pos);
        L.tile_ent.push_back((int)L.ent_node.size());
        tile++;
        tile_tets = 0;
        tile_nodes = 0;
        tile_list.clear();
    };
    for (int k = 0; k < m; k++) {
        const int e = order[k];
        int fresh = 0;
        for (int a = 0; a < 4; a++) {
            const int v = tets[4 * e + a];
            if (stamp[v] != tile) fresh++;
        }
        if (tile_tets == max_tets || tile_nodes + fresh > max_nodes) close_tile();
        for (int a = 0; a < 4; a++) {
            const int v = tets[4 * e + a];
            if (stamp[v] != tile) {
                stamp[v] = tile;
                tile_list.push_back(v);
                tile_nodes++;
            }
        }
        tile_tets++;
        pos++;
    }
    if (tile_tets > 0) close_tile();
    L.ntile = tile;
    L.nent = (int)L.ent_node.size();
    L.node_ent_off.assign(n + 1, 0);
    for (int v : L.ent_node) L.node_ent_off[v + 1]++;
    for (int i = 0; i < n; i++) L.node_ent_off[i + 1] += L.node_ent_off[i];
    L.node_ent.assign(L.nent, 0);
    std::vector<int> fill(n, 0);
    for (int q = 0; q < L.nent; q++) {
        const int v = L.ent_node[q];
        L.node_ent[L.node_ent_off[v] + fill[v]++] = q;
    }
}

// Incident (tet, slot) pairs of every tile entry, for the deterministic
// accumulation of tile partials: entry e's pairs are inc[off[e] .. off[e+1]),
// coded (tet position within the tile << 2) | slot, in ascending tet order.
inline void build_incidence(const HostLayout &L, std::vector<int> &off, std::vector<uint16_t> &inc) {
    off.assign(L.nent + 1, 0);
    inc.assign(4 * (size_t)L.m, 0);
    for (int t = 0; t < L.ntile; t++) {
        const int e0 = L.tile_ent[t];
        for (int k = L.tile_tet[t]; k < L.tile_tet[t + 1]; k++)
            for (int a = 0; a < 4; a++) off[e0 + ((L.tet_loc[k] >> (8 * a)) & 0xff) + 1]++;
    }
    for (int e = 0; e < L.nent; e++) off[e + 1] += off[e];
    std::vector<int> fill(off.begin(), off.end() - 1);
    for (int t = 0; t < L.ntile; t++) {
        const int e0 = L.tile_ent[t], k0 = L.tile_tet[t];
        for (int k = k0; k < L.tile_tet[t + 1]; k++)
            for (int a = 0; a < 4; a++)
                inc[fill[e0 + ((L.tet_loc[k] >> (8 * a)) & 0xff)]++] = (uint16_t)(((k - k0) << 2) | a);
    }
}

}  // namespace fem_layout
