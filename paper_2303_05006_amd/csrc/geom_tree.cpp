// Host-side setup: RWG edges, the adaptive octree (Section 3.4.1), neighbour
// and interaction lists, and near-field source cells (Program 2).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <unordered_map>

#include "tdbem_internal.h"

namespace tdbem {

// ------------------------------------------------------------------ mesh
void build_mesh(const tdbem_mesh *m, HostMesh &H) {
    TD_REQUIRE(m && m->xyz && m->tri && m->n_vertices >= 4 && m->n_triangles >= 4, TDBEM_EINVAL,
               "mesh: need at least 4 vertices and 4 triangles");
    TD_REQUIRE(m->n_triangles < (1ll << 30), TDBEM_EINVAL, "mesh: too many triangles");
    H.nv = (int)m->n_vertices;
    H.nt = (int)m->n_triangles;
    H.xyz.assign(m->xyz, m->xyz + 3 * (size_t)H.nv);
    H.tri.assign(m->tri, m->tri + 3 * (size_t)H.nt);
    for (int v : H.tri) TD_REQUIRE(v >= 0 && v < H.nv, TDBEM_EINVAL, "mesh: vertex index out of range");
    // directed edges: (lo, hi) traversed lo->hi belongs to T+, hi->lo to T-
    struct Half { int t, w; };
    std::vector<std::pair<uint64_t, Half>> plus, minus;
    plus.reserve(3 * (size_t)H.nt / 2 + 1);
    minus.reserve(3 * (size_t)H.nt / 2 + 1);
    for (int t = 0; t < H.nt; ++t) {
        for (int k = 0; k < 3; ++k) {
            int u = H.tri[3 * t + k], v = H.tri[3 * t + (k + 1) % 3], w = H.tri[3 * t + (k + 2) % 3];
            TD_REQUIRE(u != v, TDBEM_EINVAL, "mesh: degenerate triangle");
            uint64_t key = ((uint64_t)std::min(u, v) << 32) | (uint32_t)std::max(u, v);
            if (u < v) plus.push_back({key, {t, w}});
            else minus.push_back({key, {t, w}});
        }
    }
    auto cmp = [](const std::pair<uint64_t, Half> &a, const std::pair<uint64_t, Half> &b) { return a.first < b.first; };
    std::sort(plus.begin(), plus.end(), cmp);
    std::sort(minus.begin(), minus.end(), cmp);
    TD_REQUIRE(plus.size() == minus.size(), TDBEM_EINVAL, "mesh: not closed or not consistently oriented");
    H.ne = (int)plus.size();
    H.edge_v.resize(2 * (size_t)H.ne);
    H.etri.resize(2 * (size_t)H.ne);
    H.efree.resize(2 * (size_t)H.ne);
    H.elen.resize(H.ne);
    for (int e = 0; e < H.ne; ++e) {
        TD_REQUIRE(plus[e].first == minus[e].first && (e == 0 || plus[e].first != plus[e - 1].first),
                   TDBEM_EINVAL, "mesh: not a closed 2-manifold with consistent orientation");
        int lo = (int)(plus[e].first >> 32), hi = (int)(plus[e].first & 0xffffffffu);
        H.edge_v[2 * e] = lo;
        H.edge_v[2 * e + 1] = hi;
        H.etri[2 * e] = plus[e].second.t;
        H.etri[2 * e + 1] = minus[e].second.t;
        H.efree[2 * e] = plus[e].second.w;
        H.efree[2 * e + 1] = minus[e].second.w;
        double d2 = 0;
        for (int c = 0; c < 3; ++c) {
            double dd = H.xyz[3 * hi + c] - H.xyz[3 * lo + c];
            d2 += dd * dd;
        }
        H.elen[e] = std::sqrt(d2);
    }
    // triangle -> edges, areas, normals, 3-point rule points (2/3, 1/6, 1/6)
    H.tedge.assign(3 * (size_t)H.nt, -1);
    for (int e = 0; e < H.ne; ++e) {
        for (int s = 0; s < 2; ++s) {
            int t = H.etri[2 * e + s];
            for (int k = 0; k < 3; ++k) {
                int u = H.tri[3 * t + k], v = H.tri[3 * t + (k + 1) % 3];
                if (std::min(u, v) == H.edge_v[2 * e] && std::max(u, v) == H.edge_v[2 * e + 1]) H.tedge[3 * t + k] = e;
            }
        }
    }
    H.area.resize(H.nt);
    H.nrm.resize(3 * (size_t)H.nt);
    H.qpt.resize(9 * (size_t)H.nt);
    for (int t = 0; t < H.nt; ++t) {
        const double *a = &H.xyz[3 * H.tri[3 * t]], *b = &H.xyz[3 * H.tri[3 * t + 1]], *c = &H.xyz[3 * H.tri[3 * t + 2]];
        double e1[3], e2[3], n[3];
        for (int k = 0; k < 3; ++k) { e1[k] = b[k] - a[k]; e2[k] = c[k] - a[k]; }
        n[0] = e1[1] * e2[2] - e1[2] * e2[1];
        n[1] = e1[2] * e2[0] - e1[0] * e2[2];
        n[2] = e1[0] * e2[1] - e1[1] * e2[0];
        double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        TD_REQUIRE(nn > 0, TDBEM_EINVAL, "mesh: zero-area triangle");
        H.area[t] = 0.5 * nn;
        for (int k = 0; k < 3; ++k) H.nrm[3 * t + k] = n[k] / nn;
        const double *P[3] = {a, b, c};
        for (int q = 0; q < 3; ++q)
            for (int k = 0; k < 3; ++k) {
                double s = 0;
                for (int v = 0; v < 3; ++v) s += (v == q ? 2.0 / 3.0 : 1.0 / 6.0) * P[v][k];
                H.qpt[9 * t + 3 * q + k] = s;
            }
    }
}

// ------------------------------------------------------------------ octree
static const int LCAP = 20;  // finest integer resolution of edge midpoints

static uint64_t spread3(uint64_t x) {
    x &= 0x1fffff;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

void build_tree(const HostMesh &H, int leaf_max, int min_level, Tree &T) {
    TD_REQUIRE(leaf_max >= 1, TDBEM_EINVAL, "leaf_max must be >= 1");
    // root: tight cube around the vertices
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int v = 0; v < H.nv; ++v)
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], H.xyz[3 * v + k]);
            hi[k] = std::max(hi[k], H.xyz[3 * v + k]);
        }
    double side = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    TD_REQUIRE(side > 0, TDBEM_EINVAL, "mesh: zero extent");
    T.side = side;
    for (int k = 0; k < 3; ++k) T.origin[k] = 0.5 * (lo[k] + hi[k]) - 0.5 * side;
    // edge midpoints -> integer coordinates at LCAP; cell index at level l is
    // floor(((m - origin)/side) 2^l) clamped, the same as shifting the LCAP index
    int ne = H.ne;
    std::vector<uint32_t> q(3 * (size_t)ne);
    std::vector<std::pair<uint64_t, int>> key(ne);
    const uint32_t qmax = (1u << LCAP) - 1;
    for (int e = 0; e < ne; ++e) {
        uint64_t code = 0;
        for (int k = 0; k < 3; ++k) {
            double mid = 0.5 * (H.xyz[3 * H.edge_v[2 * e] + k] + H.xyz[3 * H.edge_v[2 * e + 1] + k]);
            double x = (mid - T.origin[k]) / side;
            double f = std::floor(x * (double)(1u << LCAP));
            uint32_t qi = f < 0 ? 0u : (f > qmax ? qmax : (uint32_t)f);
            q[3 * e + k] = qi;
            code |= spread3(qi) << (2 - k);
        }
        key[e] = {code, e};
    }
    std::sort(key.begin(), key.end());
    T.perm.resize(ne);
    T.iperm.resize(ne);
    for (int p = 0; p < ne; ++p) {
        T.perm[p] = key[p].second;
        T.iperm[key[p].second] = p;
    }
    // recursive subdivision over contiguous Morton ranges
    T.lev.clear();
    T.lev.resize(1);
    struct Node { int level, b, e, parent; };
    std::vector<Node> cur = {{0, 0, ne, -1}};
    int level = 0;
    while (!cur.empty()) {
        Level &L = T.lev[level];
        std::vector<Node> next;
        for (const Node &nd : cur) {
            int idx = L.n++;
            uint32_t cq[3];
            for (int k = 0; k < 3; ++k) cq[k] = level == 0 ? 0 : (q[3 * key[nd.b].second + k] >> (LCAP - level));
            L.ix.push_back(cq[0]); L.iy.push_back(cq[1]); L.iz.push_back(cq[2]);
            L.parent.push_back(nd.parent);
            L.ebeg.push_back(nd.b);
            L.eend.push_back(nd.e);
            bool split = (nd.e - nd.b > leaf_max || level < min_level) && level < LCAP;
            L.leaf.push_back(split ? 0 : 1);
            L.child_beg.push_back((int)next.size());
            if (split) {
                int shift = 3 * (LCAP - level - 1);
                int b = nd.b;
                while (b < nd.e) {
                    uint64_t oct = (key[b].first >> shift) & 7;
                    int e = b;
                    while (e < nd.e && ((key[e].first >> shift) & 7) == oct) ++e;
                    next.push_back({level + 1, b, e, idx});
                    b = e;
                }
            }
            L.child_end.push_back((int)next.size());
        }
        if (next.empty()) break;
        ++level;
        T.lev.resize(level + 1);
        cur.swap(next);
    }
    T.lmax = (int)T.lev.size() - 1;
    // per-edge leaf cell
    T.edge_leaf_level.assign(ne, -1);
    T.edge_leaf_cell.assign(ne, -1);
    for (int l = 0; l <= T.lmax; ++l) {
        Level &L = T.lev[l];
        for (int c = 0; c < L.n; ++c)
            if (L.leaf[c])
                for (int p = L.ebeg[c]; p < L.eend[c]; ++p) {
                    T.edge_leaf_level[p] = l;
                    T.edge_leaf_cell[p] = c;
                }
    }
    // neighbour lists (Chebyshev distance <= 1, same level, incl. self)
    for (int l = 0; l <= T.lmax; ++l) {
        Level &L = T.lev[l];
        std::unordered_map<uint64_t, int> at;
        at.reserve(2 * L.n + 1);
        auto pack = [](int x, int y, int z) { return ((uint64_t)(uint32_t)x << 42) | ((uint64_t)(uint32_t)y << 21) | (uint32_t)z; };
        for (int c = 0; c < L.n; ++c) at[pack(L.ix[c], L.iy[c], L.iz[c])] = c;
        L.nbr_off.assign(1, 0);
        L.nbr.clear();
        for (int c = 0; c < L.n; ++c) {
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        int x = L.ix[c] + dx, y = L.iy[c] + dy, z = L.iz[c] + dz;
                        if (x < 0 || y < 0 || z < 0) continue;
                        auto it = at.find(pack(x, y, z));
                        if (it != at.end()) L.nbr.push_back(it->second);
                    }
            L.nbr_off.push_back((int)L.nbr.size());
        }
    }
    // interaction lists: children of the parent's neighbours that do not touch
    for (int l = 0; l <= T.lmax; ++l) {
        Level &L = T.lev[l];
        L.il_off.assign(1, 0);
        L.il_src.clear();
        L.il_code.clear();
        for (int c = 0; c < L.n; ++c) {
            if (l >= 2) {
                const Level &P = T.lev[l - 1];
                int par = L.parent[c];
                for (int k = P.nbr_off[par]; k < P.nbr_off[par + 1]; ++k) {
                    int pn = P.nbr[k];
                    for (int s = P.child_beg[pn]; s < P.child_end[pn]; ++s) {
                        int dx = L.ix[s] - L.ix[c], dy = L.iy[s] - L.iy[c], dz = L.iz[s] - L.iz[c];
                        if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
                        L.il_src.push_back(s);
                        L.il_code.push_back(((dx + 3) * 7 + (dy + 3)) * 7 + (dz + 3));
                    }
                }
            }
            L.il_off.push_back((int)L.il_src.size());
        }
    }
}

// Program 2: for the leaf O at `level`, near sources are all edges of the
// cells in N(O) at that level, plus, for every ancestor A at a coarser level
// (>= 2), the edges of the leaf cells in N(A).
void near_source_cells(const Tree &T, int level, int cell, std::vector<std::pair<int, int>> &out) {
    out.clear();
    const Level &L = T.lev[level];
    for (int k = L.nbr_off[cell]; k < L.nbr_off[cell + 1]; ++k) out.push_back({level, L.nbr[k]});
    int c = cell;
    for (int l = level - 1; l >= 2; --l) {
        c = T.lev[l + 1].parent[c];
        const Level &A = T.lev[l];
        for (int k = A.nbr_off[c]; k < A.nbr_off[c + 1]; ++k)
            if (A.leaf[A.nbr[k]]) out.push_back({l, A.nbr[k]});
    }
}

}  // namespace tdbem
