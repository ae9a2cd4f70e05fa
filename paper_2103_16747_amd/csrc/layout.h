// Host construction of a mesh's tiled layout (plain C++, no device code):
// node numbering, tet order, tiles, the dealing of each tile's tets to
// wavefront lanes, and the node -> tile entry lists. The library builds it
// once per mesh; a CPU test program builds it under the address and
// undefined-behaviour sanitizers.
#pragma once

#include <algorithm>
#include <array>
#include <cstdint>
#include <thread>
#include <utility>
#include <vector>

namespace fem_layout {

// ---------------------------------------------------------------------------
// Tiled layout of one mesh (host construction).
// ---------------------------------------------------------------------------
struct HostLayout {
    int n = 0, m = 0, ntile = 0, nent = 0;
    std::vector<int> tile_tet, tile_ent, ent_node, node_ent_off, node_ent;
    std::vector<uint8_t> ent_slot;      // nent: LDS slot (local id in tet_loc) of each entry
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
//
// Dealing of a tile's tets to wavefront lanes. The tile kernels give
// consecutive tets to consecutive lanes; per vertex slot a, each lane reads
// the staged vectors of its tet's slot-a node (16 bytes per entry) and adds
// its nodal vector into the FP64 partials (24 bytes per entry). The LDS
// serves such an instruction 16 lanes at a time; within those 16 lanes, two
// entries whose local ids agree mod 16 (their "residue") share banks and
// cost one more pass (measured on gfx950: a 16-B read takes about 5 cycles
// per wavefront without such repeats and 12 with random ids, a 64-bit atomic
// add 8 and 26). So each tile is dealt to make every group of 16 positions
// hold, in every slot, 16 different residues:
//  1. local ids are renumbered so the 16 residue classes (ids r, r+16, ...)
//     carry nearly equal numbers of tet incidences;
//  2. tets are split into groups of 16 positions in which each residue
//     occurs at most 4 times (64 incidences over 16 residues): a greedy
//     placement, then swaps aimed at the groups that exceed it;
//  3. within a group the tets x residues multigraph has degree 4 on both
//     sides, so it splits into 4 perfect matchings (Konig's edge-colouring
//     theorem); matching c gives each tet's vertex for slot c, which fixes
//     the tet's vertex order (any of the 24: the rest constants take |det|).
// A group that keeps a residue above 4 falls back to a best-effort colouring.
inline constexpr int kPerm24[24][4] = {
    {0, 1, 2, 3}, {0, 1, 3, 2}, {0, 2, 1, 3}, {0, 2, 3, 1}, {0, 3, 1, 2}, {0, 3, 2, 1}, {1, 0, 2, 3}, {1, 0, 3, 2},
    {1, 2, 0, 3}, {1, 2, 3, 0}, {1, 3, 0, 2}, {1, 3, 2, 0}, {2, 0, 1, 3}, {2, 0, 3, 1}, {2, 1, 0, 3}, {2, 1, 3, 0},
    {2, 3, 0, 1}, {2, 3, 1, 0}, {3, 0, 1, 2}, {3, 0, 2, 1}, {3, 1, 0, 2}, {3, 1, 2, 0}, {3, 2, 0, 1}, {3, 2, 1, 0}};

inline int perm24_index(const int p[4]) {
    for (int r = 0; r < 24; r++)
        if (kPerm24[r][0] == p[0] && kPerm24[r][1] == p[1] && kPerm24[r][2] == p[2] && kPerm24[r][3] == p[3]) return r;
    return 0;
}

// Swap rounds of step 2 per tile (each moves at most one pair of tets).
constexpr int kDealSwapRounds = 1000;

// words: per tet of the tile its 4 local ids (8 bits each, ascending-node
// numbering), ne entries. Out: newid[l] = new local id of entry l;
// placed[pos] = tet * 32 + vertex order (device vertex a is the tet's
// vertex kPerm24[order][a]). Returns the incidences left above 4 per group
// and residue (0: every slot of every group is free of repeats).
inline int deal_tile(const std::vector<uint32_t> &words, int ne, std::vector<int> &newid, std::vector<int> &placed,
                     uint32_t seed) {
    const int nk = (int)words.size();
    uint64_t rs_state = 0x9E3779B97F4A7C15ull * (seed + 1);
    auto rnd = [&rs_state](uint32_t bound) {   // splitmix64 step
        uint64_t z = (rs_state += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return (uint32_t)((z ^ (z >> 31)) % bound);
    };
    std::vector<std::array<int, 4>> loc(nk);
    std::vector<int> w(ne, 0);
    for (int k = 0; k < nk; k++)
        for (int a = 0; a < 4; a++) {
            loc[k][a] = (int)((words[k] >> (8 * a)) & 0xffu);
            w[loc[k][a]]++;
        }
    const int nq = (nk + 15) / 16;
    auto cap = [&](int q) { return q == nq - 1 ? nk - 16 * (nq - 1) : 16; };
    auto lim = [&](int q) { return (4 * cap(q) + 15) / 16; };
    int limsum = 0;
    for (int q = 0; q < nq; q++) limsum += lim(q);
    // 1. residue classes: within each run of 16 ids, heaviest entries to the
    // lightest classes; then swaps between classes until none exceeds limsum
    std::vector<std::vector<int>> cls(16);
    std::vector<int> load(16, 0);
    for (int g = 0; 16 * g < ne; g++) {
        const int sz = std::min(16, ne - 16 * g);
        std::vector<int> idx(sz);
        for (int i = 0; i < sz; i++) idx[i] = 16 * g + i;
        std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return w[x] > w[y]; });
        bool used[16] = {false};
        for (int x : idx) {
            int br = -1;
            for (int r = 0; r < sz; r++)
                if (!used[r] && (br < 0 || load[r] < load[br])) br = r;
            used[br] = true;
            load[br] += w[x];
            cls[br].push_back(x);
        }
    }
    for (int step = 0; step < 4 * ne; step++) {
        int h = 0;
        for (int r = 1; r < 16; r++)
            if (load[r] > load[h]) h = r;
        if (load[h] <= limsum) break;
        int best = 0, bx = -1, by = -1, br = -1;
        for (int r = 0; r < 16; r++) {
            if (r == h) continue;
            for (size_t xi = 0; xi < cls[h].size(); xi++)
                for (size_t yi = 0; yi < cls[r].size(); yi++) {
                    const int d = w[cls[h][xi]] - w[cls[r][yi]];
                    if (d <= 0) continue;
                    const int gain = (load[h] - limsum) - std::max(0, load[h] - d - limsum) - std::max(0, load[r] + d - limsum);
                    if (gain > best) {
                        best = gain;
                        bx = (int)xi;
                        by = (int)yi;
                        br = r;
                    }
                }
        }
        if (best <= 0) break;
        const int d = w[cls[h][bx]] - w[cls[br][by]];
        std::swap(cls[h][bx], cls[br][by]);
        load[h] -= d;
        load[br] += d;
    }
    newid.assign(ne, 0);
    std::vector<int> resid(ne, 0);
    for (int r = 0; r < 16; r++) {
        std::sort(cls[r].begin(), cls[r].end());
        for (size_t i = 0; i < cls[r].size(); i++) {
            newid[cls[r][i]] = r + 16 * (int)i;
            resid[cls[r][i]] = r;
        }
    }
    // 2. groups of 16 positions with at most lim(q) incidences per residue
    std::vector<std::array<int, 4>> res(nk);
    for (int k = 0; k < nk; k++)
        for (int a = 0; a < 4; a++) res[k][a] = resid[loc[k][a]];
    std::vector<int> ord(nk);
    std::vector<long long> key(nk, 0);
    for (int k = 0; k < nk; k++) {
        ord[k] = k;
        for (int a = 0; a < 4; a++) key[k] += (long long)load[res[k][a]] * load[res[k][a]];
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return key[x] > key[y]; });
    std::vector<int> group(nk, 0), cnt(16 * (size_t)nq, 0);
    std::vector<std::vector<int>> mem(nq);
    for (int k : ord) {
        int bq = -1, bc = 1 << 30;
        for (int q = 0; q < nq; q++) {
            if ((int)mem[q].size() == cap(q)) continue;
            int c = 0, tmp[16] = {0};
            for (int a = 0; a < 4; a++) {
                const int r = res[k][a];
                c += 64 * std::max(0, cnt[16 * q + r] + ++tmp[r] - lim(q)) + cnt[16 * q + r];
            }
            if (c < bc || (c == bc && mem[q].size() < mem[bq].size())) {
                bc = c;
                bq = q;
            }
        }
        group[k] = bq;
        mem[bq].push_back(k);
        for (int a = 0; a < 4; a++) cnt[16 * bq + res[k][a]]++;
    }
    auto over = [&](int q, int r) { return std::max(0, cnt[16 * q + r] - lim(q)); };
    auto swap_change = [&](int i, int j) {   // change of the excess if tets i and j trade groups
        const int qi = group[i], qj = group[j];
        int r8[8], d8[8], n8 = 0;           // residue, change of its count in qi (qj: the opposite)
        auto add = [&](int r, int d) {
            for (int x = 0; x < n8; x++)
                if (r8[x] == r) {
                    d8[x] += d;
                    return;
                }
            r8[n8] = r;
            d8[n8++] = d;
        };
        for (int a = 0; a < 4; a++) {
            add(res[i][a], -1);
            add(res[j][a], +1);
        }
        int dl = 0;
        for (int x = 0; x < n8; x++) {
            if (!d8[x]) continue;
            const int ci = cnt[16 * qi + r8[x]], cj = cnt[16 * qj + r8[x]];
            dl += std::max(0, ci + d8[x] - lim(qi)) - std::max(0, ci - lim(qi));
            dl += std::max(0, cj - d8[x] - lim(qj)) - std::max(0, cj - lim(qj));
        }
        return dl;
    };
    int excess = 0;
    for (int q = 0; q < nq; q++)
        for (int r = 0; r < 16; r++) excess += over(q, r);
    std::vector<std::pair<int, int>> viol;
    for (int round = 0; round < kDealSwapRounds && excess > 0; round++) {
        viol.clear();
        for (int q = 0; q < nq; q++)
            for (int r = 0; r < 16; r++)
                if (over(q, r) > 0) viol.push_back({q, r});
        const std::pair<int, int> v = viol[rnd((uint32_t)viol.size())];
        // a tet of the group holding the residue, traded for one elsewhere
        // holding it fewer times: the first that lowers the excess, else a
        // random one of the best that keeps it
        int best = 1, bi = -1, bj = -1, ties = 0;
        const int j0 = (int)rnd((uint32_t)nk);
        for (int i : mem[v.first]) {
            int hi = 0;
            for (int a = 0; a < 4; a++) hi += res[i][a] == v.second;
            if (!hi) continue;
            for (int jj = 0; jj < nk && best >= 0; jj++) {
                const int j = jj + j0 < nk ? jj + j0 : jj + j0 - nk;
                if (group[j] == v.first) continue;
                int hj = 0;
                for (int a = 0; a < 4; a++) hj += res[j][a] == v.second;
                if (hj >= hi) continue;
                const int d = swap_change(i, j);
                if (d < best) {
                    best = d;
                    bi = i;
                    bj = j;
                    ties = 1;
                } else if (d == best && rnd((uint32_t)++ties) == 0) {
                    bi = i;
                    bj = j;
                }
            }
            if (best < 0) break;
        }
        if (bi < 0 || best > 0) continue;
        const int qi = group[bi], qj = group[bj];
        excess += best;
        for (int a = 0; a < 4; a++) {
            cnt[16 * qi + res[bi][a]]--;
            cnt[16 * qj + res[bi][a]]++;
            cnt[16 * qj + res[bj][a]]--;
            cnt[16 * qi + res[bj][a]]++;
        }
        group[bi] = qj;
        group[bj] = qi;
        std::replace(mem[qi].begin(), mem[qi].end(), bi, bj);
        std::replace(mem[qj].begin(), mem[qj].end(), bj, bi);
    }
    // 3. per group: slot c of each tet = colour c of a 4-edge-colouring of the
    // tets x residues multigraph, by alternating-path recolouring; the
    // colours of a group are then renamed (one of the 24 orders) so that as
    // few of its nodes as possible take a slot in which an earlier group of
    // the same wavefront (4 groups) already has them: lanes of one atomic
    // instruction that add into the same address are serialised
    placed.assign(nk, 0);
    std::vector<std::pair<int, int>> path;
    std::array<std::vector<char>, 4> used;
    for (int q = 0; q < nq; q++) {
        if (q % 4 == 0)
            for (auto &u : used) u.assign(ne, 0);
        const std::vector<int> &M = mem[q];
        const int nt = (int)M.size();
        std::vector<std::array<int, 4>> slot(nt), at_t(nt);   // slot of (tet, vertex); vertex of (tet, colour)
        std::array<std::array<int, 4>, 16> at_rt, at_rv;       // (tet, vertex) of (residue, colour)
        for (auto &x : slot) x.fill(-1);
        for (auto &x : at_t) x.fill(-1);
        for (auto &x : at_rt) x.fill(-1);
        for (auto &x : at_rv) x.fill(-1);
        for (int t = 0; t < nt; t++)
            for (int a = 0; a < 4; a++) {
                const int r = res[M[t]][a];
                int al = -1, be = -1;
                for (int c = 0; c < 4 && al < 0; c++)
                    if (at_t[t][c] < 0) al = c;
                for (int c = 0; c < 4 && be < 0; c++)
                    if (at_rt[r][c] < 0) be = c;
                if (be >= 0 && at_rt[r][al] >= 0) {
                    // colour al is taken at r, be is free there: swap al and
                    // be along the path r -al- t1 -be- r2 -al- ..., which
                    // cannot reach tet t (al is free at t)
                    path.clear();
                    int cr = r;
                    while ((int)path.size() < 8 * nt) {
                        const int t1 = at_rt[cr][al];
                        if (t1 < 0) break;
                        path.push_back({t1, at_rv[cr][al]});
                        const int a2 = at_t[t1][be];
                        if (a2 < 0) break;
                        path.push_back({t1, a2});   // t1's two edges trade colours
                        cr = res[M[t1]][a2];
                        if (at_rt[cr][be] != t1 || at_rv[cr][be] != a2) break;   // edge of an over-full residue
                    }
                    for (const auto &e : path) {
                        const int c = slot[e.first][e.second], rr = res[M[e.first]][e.second];
                        at_t[e.first][c] = -1;
                        if (at_rt[rr][c] == e.first && at_rv[rr][c] == e.second) at_rt[rr][c] = at_rv[rr][c] = -1;
                    }
                    for (const auto &e : path) {
                        const int c = slot[e.first][e.second] == al ? be : al, rr = res[M[e.first]][e.second];
                        slot[e.first][e.second] = c;
                        at_t[e.first][c] = e.second;
                        if (at_rt[rr][c] < 0) {
                            at_rt[rr][c] = e.first;
                            at_rv[rr][c] = e.second;
                        }
                    }
                }
                slot[t][a] = al;
                at_t[t][al] = a;
                if (at_rt[r][al] < 0) {
                    at_rt[r][al] = t;
                    at_rv[r][al] = a;
                }
            }
        int best_r = 0, best_c = 1 << 30;
        for (int r = 0; r < 24; r++) {
            int c = 0;
            for (int t = 0; t < nt; t++)
                for (int a = 0; a < 4; a++)
                    if (slot[t][a] >= 0) c += used[kPerm24[r][slot[t][a]]][loc[M[t]][a]];
            if (c < best_c) {
                best_c = c;
                best_r = r;
            }
        }
        for (int t = 0; t < nt; t++)
            for (int a = 0; a < 4; a++)
                if (slot[t][a] >= 0) {
                    slot[t][a] = kPerm24[best_r][slot[t][a]];
                    used[slot[t][a]][loc[M[t]][a]] = 1;
                }
        for (int t = 0; t < nt; t++) {
            int p[4] = {-1, -1, -1, -1};
            for (int a = 0; a < 4; a++)
                if (slot[t][a] >= 0 && slot[t][a] < 4) p[slot[t][a]] = a;
            const bool perm = p[0] >= 0 && p[1] >= 0 && p[2] >= 0 && p[3] >= 0;
            placed[16 * q + t] = M[t] * 32 + (perm ? perm24_index(p) : 0);
        }
    }
    return excess;
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
    // tiles: consecutive tets of the Morton order, cut at max_tets tets or
    // max_nodes distinct nodes; each tile's nodes in ascending order
    std::vector<int> stamp(n, -1);
    std::vector<std::vector<int>> tnodes;
    L.tile_tet.assign(1, 0);
    int tile = 0, tile_tets = 0;
    std::vector<int> cur;
    for (int k = 0; k < m; k++) {
        const int e = order[k];
        int fresh = 0;
        for (int a = 0; a < 4; a++) fresh += stamp[tets[4 * (size_t)e + a]] != tile;
        if (tile_tets == max_tets || (int)cur.size() + fresh > max_nodes) {
            std::sort(cur.begin(), cur.end());
            tnodes.push_back(cur);
            L.tile_tet.push_back(k);
            cur.clear();
            tile++;
            tile_tets = 0;
        }
        for (int a = 0; a < 4; a++) {
            const int v = tets[4 * (size_t)e + a];
            if (stamp[v] != tile) {
                stamp[v] = tile;
                cur.push_back(v);
            }
        }
        tile_tets++;
    }
    if (tile_tets > 0) {
        std::sort(cur.begin(), cur.end());
        tnodes.push_back(cur);
        L.tile_tet.push_back(m);
        tile++;
    }
    L.ntile = tile;
    L.tile_ent.assign(L.ntile + 1, 0);
    for (int t = 0; t < L.ntile; t++) L.tile_ent[t + 1] = L.tile_ent[t] + (int)tnodes[t].size();
    L.nent = L.tile_ent[L.ntile];
    L.ent_node.assign(L.nent, 0);
    L.ent_slot.assign(L.nent, 0);
    L.tet_loc.assign(m, 0);
    L.order.assign(m, 0);
    L.tet_nodes.assign(4 * (size_t)m, 0);
    // dealing, tile by tile (independent; spread over host threads, each
    // tile's pseudo-random choices seeded by its index)
    auto deal_one = [&](int t) {
        const std::vector<int> &nodes = tnodes[t];
        const int k0 = L.tile_tet[t], k1 = L.tile_tet[t + 1], e0 = L.tile_ent[t], ne = (int)nodes.size();
        std::vector<uint32_t> words(k1 - k0);
        for (int k = k0; k < k1; k++) {
            const int e = order[k];
            uint32_t w = 0;
            for (int a = 0; a < 4; a++) {
                const int v = tets[4 * (size_t)e + a];
                const int l = (int)(std::lower_bound(nodes.begin(), nodes.end(), v) - nodes.begin());
                w |= (uint32_t)l << (8 * a);
            }
            words[k - k0] = w;
        }
        std::vector<int> newid, placed;
        deal_tile(words, ne, newid, placed, (uint32_t)t);
        // entries stay in ascending node order (the node pass reads a
        // node's partials at consecutive addresses); slots follow the dealing
        for (int l = 0; l < ne; l++) {
            L.ent_node[e0 + l] = nodes[l];
            L.ent_slot[e0 + l] = (uint8_t)newid[l];
        }
        for (int k = k0; k < k1; k++) {
            const int src = placed[k - k0] >> 5, r = placed[k - k0] & 31;
            const int e = order[k0 + src];
            uint32_t w = 0;
            for (int a = 0; a < 4; a++) {
                const int from = kPerm24[r][a];
                w |= (uint32_t)newid[(words[src] >> (8 * from)) & 0xffu] << (8 * a);
                L.tet_nodes[4 * (size_t)k + a] = tets[4 * (size_t)e + from];
            }
            L.tet_loc[k] = w;
            L.order[k] = e;
        }
    };
    const int hw = (int)std::thread::hardware_concurrency();
    const int nth = std::max(1, std::min({hw > 0 ? hw : 1, 16, L.ntile}));
    if (nth == 1) {
        for (int t = 0; t < L.ntile; t++) deal_one(t);
    } else {
        std::vector<std::thread> pool;
        for (int i = 0; i < nth; i++)
            pool.emplace_back([&, i]() {
                for (int t = i; t < L.ntile; t += nth) deal_one(t);
            });
        for (std::thread &th : pool) th.join();
    }
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
    std::vector<int> ent_of(256, 0);   // tile entry of each LDS slot
    for (int pass = 0; pass < 2; pass++) {
        std::vector<int> fill;
        if (pass == 1) {
            for (int e = 0; e < L.nent; e++) off[e + 1] += off[e];
            fill.assign(off.begin(), off.end() - 1);
        }
        for (int t = 0; t < L.ntile; t++) {
            const int e0 = L.tile_ent[t], k0 = L.tile_tet[t];
            for (int e = e0; e < L.tile_ent[t + 1]; e++) ent_of[L.ent_slot[e]] = e;
            for (int k = k0; k < L.tile_tet[t + 1]; k++)
                for (int a = 0; a < 4; a++) {
                    const int e = ent_of[(L.tet_loc[k] >> (8 * a)) & 0xff];
                    if (pass == 0)
                        off[e + 1]++;
                    else
                        inc[fill[e]++] = (uint16_t)(((k - k0) << 2) | a);
                }
        }
    }
}

// Order of `heavy` blocks 0..heavy-1 and `light` blocks heavy..heavy+light-1
// with the light ones spread evenly among the heavy ones (block h sits at
// (h + 1/2) / heavy of the way, block l at (l + 1/2) / light). Each XCD runs
// a contiguous share of a work table (blocks are dealt to the XCDs
// round-robin and renumbered so that consecutive work items share one); in
// plain index order the light blocks (the contact blocks of the tile pass;
// the node blocks holding only fixed nodes, which a CG update skips) would
// all fall to the last XCDs, which then idle while the others carry the
// heavy work.
inline std::vector<int> spread_order(int heavy, int light) {
    std::vector<int> o;
    o.reserve(heavy + light);
    int h = 0, l = 0;
    while (h < heavy || l < light) {
        const bool take_light =
            l < light && (h >= heavy || (2LL * l + 1) * heavy < (2LL * h + 1) * light);
        o.push_back(take_light ? heavy + l++ : h++);
    }
    return o;
}

}  // namespace fem_layout
