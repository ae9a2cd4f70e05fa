// CPU check of the host layout construction (paper_2103_16747_amd/csrc/layout.h),
// built by tests/test_sanitizers.py with the address and undefined-behaviour
// sanitizers. Reads a mesh (int32 n, int32 m, n x 3 doubles, m x 4 int32) from
// the file named by argv[1], builds the node numbering and the tiled layout
// with the limits argv[2] (tets per tile) and argv[3] (nodes per tile), and
// checks every invariant the device kernels rely on. Prints one line
// "ok tiles=<T> entries=<E>" and exits 0, or names the first broken
// invariant and exits 1.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_2103_16747_amd/csrc/layout.h"

using namespace fem_layout;

static int bad(const char *what, long long a, long long b) {
    std::printf("FAIL %s (%lld, %lld)\n", what, a, b);
    return 1;
}

static double det_dm(const double *X, const int *t) {
    double D[9];
    for (int a = 0; a < 3; a++)
        for (int i = 0; i < 3; i++) D[3 * i + a] = X[3 * t[a + 1] + i] - X[3 * t[0] + i];
    return D[0] * (D[4] * D[8] - D[5] * D[7]) - D[1] * (D[3] * D[8] - D[5] * D[6]) +
           D[2] * (D[3] * D[7] - D[4] * D[6]);
}

int main(int argc, char **argv) {
    if (argc != 4) {
        std::fprintf(stderr, "usage: layout_check mesh.bin max_tets max_nodes\n");
        return 2;
    }
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return bad("open", 0, 0);
    int n = 0, m = 0;
    if (std::fread(&n, 4, 1, f) != 1 || std::fread(&m, 4, 1, f) != 1 || n <= 0 || m <= 0) return bad("header", n, m);
    std::vector<double> X(3 * (size_t)n);
    std::vector<int> T(4 * (size_t)m);
    if (std::fread(X.data(), 8, X.size(), f) != X.size() || std::fread(T.data(), 4, T.size(), f) != T.size())
        return bad("body", n, m);
    std::fclose(f);
    const int max_tets = std::atoi(argv[2]), max_nodes = std::atoi(argv[3]);

    // node numbering: a permutation of 0..n-1
    const std::vector<int> perm = node_order(X.data(), n, T.data(), m);
    if ((int)perm.size() != n) return bad("node_order size", (long long)perm.size(), n);
    std::vector<char> seen(n, 0);
    for (int v : perm) {
        if (v < 0 || v >= n || seen[v]) return bad("node_order not a permutation", v, n);
        seen[v] = 1;
    }
    // tet order: a permutation of 0..m-1
    const std::vector<int> order = morton_order(X.data(), n, T.data(), m);
    std::vector<char> tseen(m, 0);
    for (int e : order) {
        if (e < 0 || e >= m || tseen[e]) return bad("morton_order not a permutation", e, m);
        tseen[e] = 1;
    }

    HostLayout L;
    build_layout(X.data(), n, T.data(), m, max_tets, max_nodes, L);
    if (L.n != n || L.m != m) return bad("sizes", L.n, L.m);
    if ((int)L.tile_tet.size() != L.ntile + 1 || (int)L.tile_ent.size() != L.ntile + 1) return bad("tile arrays", L.ntile, 0);
    if (L.tile_tet[0] != 0 || L.tile_tet[L.ntile] != m) return bad("tile tet range", L.tile_tet[0], L.tile_tet[L.ntile]);
    if (L.tile_ent[0] != 0 || L.tile_ent[L.ntile] != L.nent) return bad("tile entry range", L.tile_ent[L.ntile], L.nent);
    std::fill(tseen.begin(), tseen.end(), 0);
    for (int t = 0; t < L.ntile; t++) {
        const int k0 = L.tile_tet[t], k1 = L.tile_tet[t + 1], e0 = L.tile_ent[t], e1 = L.tile_ent[t + 1];
        if (k1 <= k0 || k1 - k0 > max_tets) return bad("tets per tile", t, k1 - k0);
        if (e1 <= e0 || e1 - e0 > max_nodes) return bad("nodes per tile", t, e1 - e0);
        for (int q = e0 + 1; q < e1; q++)
            if (L.ent_node[q] <= L.ent_node[q - 1]) return bad("entries not ascending", t, q);
        // LDS slots: a permutation of 0 .. ne-1; ent_of[slot] = entry
        if ((int)L.ent_slot.size() != L.nent) return bad("slot array", (long long)L.ent_slot.size(), L.nent);
        std::vector<int> ent_of(e1 - e0, -1);
        for (int q = e0; q < e1; q++) {
            const int sl = L.ent_slot[q];
            if (sl >= e1 - e0 || ent_of[sl] >= 0) return bad("slots not a permutation", t, sl);
            ent_of[sl] = q;
        }
        for (int k = k0; k < k1; k++) {
            const int e = L.order[k];
            if (e < 0 || e >= m || tseen[e]) return bad("tile order not a permutation", k, e);
            tseen[e] = 1;
            // device vertex order: a reordering of the tet's vertices
            const int *dn = &L.tet_nodes[4 * (size_t)k];
            const int *in = &T[4 * (size_t)e];
            for (int a = 0; a < 4; a++) {
                bool found = false;
                for (int b = 0; b < 4; b++) found = found || dn[a] == in[b];
                if (!found) return bad("device vertices differ from the tet's", k, a);
                // the packed local slot names this vertex's entry in the tile
                const int slot = (int)((L.tet_loc[k] >> (8 * a)) & 0xffu);
                if (slot >= e1 - e0) return bad("local slot beyond the tile", k, slot);
                if (L.ent_node[ent_of[slot]] != dn[a]) return bad("local slot names another node", k, slot);
            }
            for (int a = 0; a < 4; a++)
                for (int b = a + 1; b < 4; b++)
                    if (dn[a] == dn[b]) return bad("device vertex repeated", k, a);
            const double d0 = det_dm(X.data(), in), d1 = det_dm(X.data(), dn);
            if (std::fabs(std::fabs(d0) - std::fabs(d1)) > 1e-9 * std::fabs(d0)) return bad("reordering changed |det D_m|", k, e);
        }
    }
    // node -> entry lists: each entry exactly once, under its own node
    if ((int)L.node_ent_off.size() != n + 1 || L.node_ent_off[n] != L.nent) return bad("node entry offsets", n, L.nent);
    std::vector<char> eseen(L.nent, 0);
    for (int v = 0; v < n; v++)
        for (int q = L.node_ent_off[v]; q < L.node_ent_off[v + 1]; q++) {
            const int ent = L.node_ent[q];
            if (ent < 0 || ent >= L.nent || eseen[ent]) return bad("node entry list", v, ent);
            if (L.ent_node[ent] != v) return bad("entry under the wrong node", v, ent);
            eseen[ent] = 1;
        }
    // incidence lists: every (tet, slot) of a tile exactly once, under the
    // entry of that slot, in ascending tet order
    std::vector<int> ioff;
    std::vector<uint16_t> inc;
    build_incidence(L, ioff, inc);
    if ((int)ioff.size() != L.nent + 1 || ioff[L.nent] != 4 * m) return bad("incidence offsets", L.nent, m);
    for (int t = 0; t < L.ntile; t++) {
        const int e0 = L.tile_ent[t], k0 = L.tile_tet[t];
        for (int e = e0; e < L.tile_ent[t + 1]; e++) {
            int last = -1;
            for (int q = ioff[e]; q < ioff[e + 1]; q++) {
                const int k = inc[q] >> 2, a = inc[q] & 3;
                if (k < last || k0 + k >= L.tile_tet[t + 1]) return bad("incidence order", e, k);
                if ((int)((L.tet_loc[k0 + k] >> (8 * a)) & 0xff) != L.ent_slot[e]) return bad("incidence slot", e, k);
                last = k;
            }
        }
    }
    // dealing: largest number of lanes sharing a residue (local id mod 16) in
    // one slot of a group of 16 consecutive positions, averaged (1 = no LDS
    // bank repeats)
    long long groups = 0, passes = 0;
    for (int t = 0; t < L.ntile; t++) {
        const int k0 = L.tile_tet[t], nk = L.tile_tet[t + 1] - k0;
        for (int q0 = 0; q0 < nk; q0 += 16)
            for (int a = 0; a < 4; a++) {
                int h[16] = {0}, mx = 0;
                for (int j = q0; j < std::min(nk, q0 + 16); j++) mx = std::max(mx, ++h[(L.tet_loc[k0 + j] >> (8 * a)) & 15]);
                groups++;
                passes += mx;
            }
    }
    // work-table column order of this mesh's tile and contact blocks (and of
    // a range of other counts): a permutation keeping each kind in ascending
    // order, with every prefix holding its proportional share of light blocks
    // to within one
    {
        const int nc_blocks = std::max(1, L.ntile / 6);
        const int cases[][2] = {{L.ntile, nc_blocks}, {1, 0}, {0, 3}, {36, 8}, {97, 15}, {5, 40}, {1, 1}, {300, 7}};
        for (const auto &c : cases) {
            const int heavy = c[0], light = c[1];
            const std::vector<int> o = spread_order(heavy, light);
            if ((int)o.size() != heavy + light) return bad("spread size", (long long)o.size(), heavy + light);
            int h = 0, l = 0;
            for (int k = 0; k < (int)o.size(); k++) {
                if (o[k] < heavy) {
                    if (o[k] != h++) return bad("spread heavy order", o[k], h - 1);
                } else if (o[k] != heavy + l++) {
                    return bad("spread light order", o[k], heavy + l - 1);
                }
                // light blocks among the first k + 1, against (k + 1) light / total
                const double share = (double)(k + 1) * light / (double)(heavy + light);
                if (std::fabs(l - share) > 1.0) return bad("spread share", l, (long long)std::lround(share));
            }
        }
    }
    std::printf("ok tiles=%d entries=%d passes=%.4f\n", L.ntile, L.nent, (double)passes / (double)groups);
    return 0;
}
