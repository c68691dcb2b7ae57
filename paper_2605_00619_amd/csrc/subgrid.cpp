// Sub-tetrahedral split, agglomerated DOFs and face pairing (Sec. 4.1).
//
// Split: each polygon face is fanned about its vertex-mean centroid F, each
// fan triangle is coned to the cell's vertex-mean centroid C, giving one
// sub-tet (a, b, F, C) per polygon edge (a, b) in the face's outward cyclic
// order; its only boundary face is (a, b, F).  Faces of a cell are visited in
// ascending global face id; an owned face in its listed corner order, a
// neighbour face in reversed corner order.
//
// Cell DOFs ("union without repetition" of the sub-tet nodes, Sec. 4.1): a
// node is identified by the sorted list of (sub-grid vertex, integer
// barycentric weight) pairs with positive weight; sub-grid vertices are
// ranked mesh vertices (by global id) < face centroids (by global face id) <
// the cell centroid.  DOFs are numbered by ascending (number of pairs, list).
// Because the identification uses global ids only, the same physical node on
// a shared face has the same key in both cells, which gives the pairing.
#include "subgrid.hpp"

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <map>
#include <thread>
#include <unordered_map>

#include "refelem.hpp"

namespace afe {
namespace {

constexpr int64_t kFaceTag = int64_t(1) << 40;
constexpr int64_t kCellTag = int64_t(2) << 40;

struct Key {
    int cnt = 0;
    int64_t id[4] = {0, 0, 0, 0};
    int w[4] = {0, 0, 0, 0};
    bool operator<(const Key &o) const {
        if (cnt != o.cnt) return cnt < o.cnt;
        for (int i = 0; i < cnt; ++i) {
            if (id[i] != o.id[i]) return id[i] < o.id[i];
            if (w[i] != o.w[i]) return w[i] < o.w[i];
        }
        return false;
    }
    bool operator==(const Key &o) const {
        if (cnt != o.cnt) return false;
        for (int i = 0; i < cnt; ++i)
            if (id[i] != o.id[i] || w[i] != o.w[i]) return false;
        return true;
    }
};

Key make_key(const int64_t ids[4], const std::array<int, 4> &bary) {
    std::array<std::pair<int64_t, int>, 4> p;
    int n = 0;
    for (int j = 0; j < 4; ++j)
        if (bary[j] > 0) p[n++] = {ids[j], bary[j]};
    std::sort(p.begin(), p.begin() + n);
    Key k;
    k.cnt = n;
    for (int i = 0; i < n; ++i) {
        k.id[i] = p[i].first;
        k.w[i] = p[i].second;
    }
    return k;
}

struct V3 {
    double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

struct CellBuild {
    afe_status status = AFE_OK;
    std::string err;
    std::vector<Key> keys;              // DOF keys in DOF order
    std::vector<int32_t> conn;          // [K][np]
    std::vector<double> geo;            // [K][10]
    std::vector<double> tri;            // [K][4]
    std::vector<int32_t> face;          // [K]
    std::vector<int32_t> ea, eb;        // [K] edge vertex ids
    std::vector<std::array<double, 3>> dof_x;
    std::vector<double> mrow;
    double h = 0.0, vol = 0.0;
};

}  // namespace

afe_status build_host_grid(const afe_mesh &mesh, int N, HostGrid &g, std::string &err) {
    if (N < 1 || N > kMaxN) {
        err = "N must be 1, 2, 3 or 4";
        return AFE_E_ARG;
    }
    if (mesh.n_cells <= 0 || mesh.n_faces <= 0 || mesh.n_vertices <= 0 || !mesh.xyz || !mesh.face_ptr ||
        !mesh.face_vtx || !mesh.face_vshift || !mesh.face_cell || !mesh.nbr_shift || !(mesh.box > 0.0)) {
        err = "incomplete mesh";
        return AFE_E_ARG;
    }
    const RefData &R = ref_data(N);
    const int np = R.np, nf = R.nf;
    const int nc = mesh.n_cells;
    const double L = mesh.box;
    g = HostGrid();
    g.N = N;
    g.np = np;
    g.nf = nf;
    g.n_cells = nc;
    g.box = L;
    // faces of each cell, ascending face id
    std::vector<std::vector<std::pair<int, int>>> cell_faces(nc);
    for (int f = 0; f < mesh.n_faces; ++f) {
        // neighbour -1: a face on the boundary of a bounded mesh
        int o = mesh.face_cell[2 * f], n = mesh.face_cell[2 * f + 1];
        if (o < 0 || o >= nc || n < -1 || n >= nc || o == n || mesh.face_ptr[f + 1] - mesh.face_ptr[f] < 3) {
            err = "face " + std::to_string(f) + " has invalid cells or fewer than 3 corners";
            return AFE_E_BAD_MESH;
        }
        cell_faces[o].push_back({f, 0});
        if (n >= 0) cell_faces[n].push_back({f, 1});
    }
    std::vector<double> mhat_colsum(np, 0.0);
    for (int m = 0; m < np; ++m)
        for (int p = 0; p < np; ++p) mhat_colsum[p] += R.M[m * np + p];

    std::vector<CellBuild> cb(nc);
    auto build_one = [&](int c) {
        CellBuild &B = cb[c];
        struct Corner {
            int v;
            V3 x;
        };
        std::vector<std::pair<int, std::vector<Corner>>> faces;
        std::map<int, V3> verts;
        for (auto [f, side] : cell_faces[c]) {
            int b0 = mesh.face_ptr[f], b1 = mesh.face_ptr[f + 1];
            std::vector<Corner> cs;
            for (int i = b0; i < b1; ++i) {
                int v = mesh.face_vtx[i];
                if (v < 0 || v >= mesh.n_vertices) {
                    B.status = AFE_E_BAD_MESH;
                    B.err = "vertex id out of range";
                    return;
                }
                double s[3];
                for (int d = 0; d < 3; ++d) {
                    double sh = double(mesh.face_vshift[3 * i + d]);
                    if (side == 1) sh -= double(mesh.nbr_shift[3 * f + d]);
                    s[d] = sh;
                }
                V3 x = {mesh.xyz[3 * v] + s[0] * L, mesh.xyz[3 * v + 1] + s[1] * L, mesh.xyz[3 * v + 2] + s[2] * L};
                cs.push_back({v, x});
            }
            if (side == 1) std::reverse(cs.begin(), cs.end());
            for (auto &cn : cs) {
                auto it = verts.find(cn.v);
                if (it == verts.end())
                    verts.emplace(cn.v, cn.x);
                else if (it->second.x != cn.x.x || it->second.y != cn.x.y || it->second.z != cn.x.z) {
                    B.status = AFE_E_BAD_MESH;
                    B.err = "cell " + std::to_string(c) + " sees vertex " + std::to_string(cn.v) + " at two positions";
                    return;
                }
            }
            faces.push_back({f, std::move(cs)});
        }
        // cell centroid: mean of the distinct vertices, ascending id
        V3 C = {0, 0, 0};
        for (auto &kv : verts) {
            C.x += kv.second.x;
            C.y += kv.second.y;
            C.z += kv.second.z;
        }
        double inv = 1.0 / double(verts.size());
        C = {C.x * inv, C.y * inv, C.z * inv};
        double hmax = 0.0;
        for (auto &a : verts)
            for (auto &b : verts) {
                V3 d = sub(a.second, b.second);
                hmax = std::max(hmax, std::sqrt(dot(d, d)));
            }
        B.h = hmax;
        // sub-tets
        struct Sub {
            int64_t ids[4];
            V3 X[4];
            int face;
        };
        std::vector<Sub> subs;
        for (auto &fc : faces) {
            const auto &cs = fc.second;
            int k = int(cs.size());
            V3 F = {0, 0, 0};
            for (auto &cn : cs) {
                F.x += cn.x.x;
                F.y += cn.x.y;
                F.z += cn.x.z;
            }
            F = {F.x / k, F.y / k, F.z / k};
            for (int e = 0; e < k; ++e) {
                const Corner &a = cs[e], &b = cs[(e + 1) % k];
                Sub s;
                s.ids[0] = a.v;
                s.ids[1] = b.v;
                s.ids[2] = kFaceTag + fc.first;
                s.ids[3] = kCellTag;
                s.X[0] = a.x;
                s.X[1] = b.x;
                s.X[2] = F;
                s.X[3] = C;
                s.face = fc.first;
                subs.push_back(s);
            }
        }
        const int K = int(subs.size());
        std::vector<Key> nk(size_t(K) * np);
        for (int k = 0; k < K; ++k)
            for (int m = 0; m < np; ++m) nk[size_t(k) * np + m] = make_key(subs[k].ids, R.bary[m]);
        std::vector<Key> uk(nk);
        std::sort(uk.begin(), uk.end());
        uk.erase(std::unique(uk.begin(), uk.end()), uk.end());
        B.keys = uk;
        const int nd = int(uk.size());
        B.conn.resize(size_t(K) * np);
        for (int k = 0; k < K; ++k)
            for (int m = 0; m < np; ++m)
                B.conn[size_t(k) * np + m] =
                    int32_t(std::lower_bound(uk.begin(), uk.end(), nk[size_t(k) * np + m]) - uk.begin());
        B.geo.resize(size_t(K) * 10);
        B.tri.resize(size_t(K) * 4);
        B.face.resize(K);
        B.ea.resize(K);
        B.eb.resize(K);
        B.dof_x.assign(nd, {0.0, 0.0, 0.0});
        B.mrow.assign(nd, 0.0);
        double vol = 0.0;
        int sign = 0;
        for (int k = 0; k < K; ++k) {
            const Sub &s = subs[k];
            V3 c1 = sub(s.X[1], s.X[0]), c2 = sub(s.X[2], s.X[0]), c3 = sub(s.X[3], s.X[0]);
            // J = [c1 | c2 | c3];  J^{-1} rows = (c2 x c3, c3 x c1, c1 x c2) / det
            V3 r0 = cross(c2, c3), r1 = cross(c3, c1), r2 = cross(c1, c2);
            double det = dot(c1, r0);
            int sg = det > 0 ? 1 : (det < 0 ? -1 : 0);
            if (sg == 0 || !std::isfinite(det) || (sign != 0 && sg != sign)) {
                B.status = AFE_E_DEGENERATE_SUBTET;
                B.err = "cell " + std::to_string(c) + " sub-tet " + std::to_string(k) + " is degenerate or inverted";
                return;
            }
            sign = sg;
            double* G = &B.geo[size_t(k) * 10];
            V3 rows[3] = {r0, r1, r2};
            for (int d = 0; d < 3; ++d) {
                G[3 * d + 0] = rows[d].x / det;
                G[3 * d + 1] = rows[d].y / det;
                G[3 * d + 2] = rows[d].z / det;
            }
            double adet = std::fabs(det);
            G[9] = adet;
            vol += adet / 6.0;
            V3 cr = cross(sub(s.X[1], s.X[0]), sub(s.X[2], s.X[0]));
            double nrm = std::sqrt(dot(cr, cr));
            double* T = &B.tri[size_t(k) * 4];
            T[0] = nrm;  // 2 * area
            T[1] = cr.x / nrm;
            T[2] = cr.y / nrm;
            T[3] = cr.z / nrm;
            B.face[k] = s.face;
            B.ea[k] = int32_t(s.ids[0]);
            B.eb[k] = int32_t(s.ids[1]);
            for (int m = 0; m < np; ++m) {
                int l = B.conn[size_t(k) * np + m];
                const auto &xi = R.xi[m];
                B.dof_x[l] = {s.X[0].x + c1.x * xi[0] + c2.x * xi[1] + c3.x * xi[2],
                              s.X[0].y + c1.y * xi[0] + c2.y * xi[1] + c3.y * xi[2],
                              s.X[0].z + c1.z * xi[0] + c2.z * xi[1] + c3.z * xi[2]};
                B.mrow[l] += adet * mhat_colsum[m];
            }
        }
        B.vol = vol;
    };
    {
        unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::atomic<int> next{0};
        std::vector<std::thread> pool;
        for (unsigned t = 0; t < nth; ++t)
            pool.emplace_back([&] {
                for (int c = next++; c < nc; c = next++) build_one(c);
            });
        for (auto &t : pool) t.join();
    }
    for (int c = 0; c < nc; ++c)
        if (cb[c].status != AFE_OK) {
            err = cb[c].err;
            return cb[c].status;
        }
    // flatten
    g.dof_ptr.assign(nc + 1, 0);
    g.sub_ptr.assign(nc + 1, 0);
    for (int c = 0; c < nc; ++c) {
        g.dof_ptr[c + 1] = g.dof_ptr[c] + int64_t(cb[c].keys.size());
        g.sub_ptr[c + 1] = g.sub_ptr[c] + int64_t(cb[c].face.size());
        g.max_cell_dofs = std::max(g.max_cell_dofs, int(cb[c].keys.size()));
        g.max_cell_subtets = std::max(g.max_cell_subtets, int(cb[c].face.size()));
    }
    g.ndof = g.dof_ptr[nc];
    g.nsub = g.sub_ptr[nc];
    if (g.nsub * np >= (int64_t(1) << 31) || g.ndof >= (int64_t(1) << 31)) {
        err = "mesh too large for 32-bit DOF indexing";
        return AFE_E_ARG;
    }
    g.conn.resize(size_t(g.nsub) * np);
    g.sub_cell.resize(g.nsub);
    g.geo.resize(size_t(g.nsub) * 10);
    g.tri.resize(size_t(g.nsub) * 4);
    g.nbr_sub.assign(g.nsub, -1);
    g.perm.assign(size_t(g.nsub) * nf, -1);
    g.h.resize(nc);
    g.vol.resize(nc);
    g.mrow.resize(g.ndof);
    g.dof_x.resize(size_t(3) * g.ndof);
    g.dof_cell.resize(g.ndof);
    g.h_min = 1e300;
    for (int c = 0; c < nc; ++c) {
        const CellBuild &B = cb[c];
        int64_t s0 = g.sub_ptr[c], d0 = g.dof_ptr[c];
        std::copy(B.conn.begin(), B.conn.end(), g.conn.begin() + s0 * np);
        std::copy(B.geo.begin(), B.geo.end(), g.geo.begin() + s0 * 10);
        std::copy(B.tri.begin(), B.tri.end(), g.tri.begin() + s0 * 4);
        for (int64_t k = s0; k < g.sub_ptr[c + 1]; ++k) g.sub_cell[k] = c;
        for (size_t l = 0; l < B.keys.size(); ++l) {
            g.mrow[d0 + l] = B.mrow[l];
            g.dof_cell[d0 + l] = c;
            for (int d = 0; d < 3; ++d) g.dof_x[size_t(d) * g.ndof + d0 + l] = B.dof_x[l][d];
        }
        g.h[c] = B.h;
        g.vol[c] = B.vol;
        g.h_min = std::min(g.h_min, B.h);
    }
    // pairing: the neighbour's sub-tet on the same triangle has the edge reversed
    std::vector<std::unordered_map<int64_t, int>> tri_of(nc);
    auto tkey = [](int f, int a, int b) { return (int64_t(f) << 42) ^ (int64_t(a) << 21) ^ int64_t(b); };
    for (int c = 0; c < nc; ++c)
        for (size_t k = 0; k < cb[c].face.size(); ++k) tri_of[c][tkey(cb[c].face[k], cb[c].ea[k], cb[c].eb[k])] = int(k);
    g.n_btri = 0;
    g.bnode_x.clear();
    for (int c = 0; c < nc; ++c) {
        const CellBuild &B = cb[c];
        for (size_t k = 0; k < B.face.size(); ++k) {
            int f = B.face[k];
            int o = mesh.face_cell[2 * f], nb = mesh.face_cell[2 * f + 1];
            int64_t gk = g.sub_ptr[c] + int64_t(k);
            if (nb < 0) {
                // boundary triangle b (ascending sub-tet order): nbr_sub = -1 - b,
                // face node j is its own partner, coordinates of its face nodes kept
                const int64_t b = g.n_btri++;
                g.nbr_sub[gk] = int32_t(-1 - b);
                for (int j = 0; j < nf; ++j) {
                    g.perm[size_t(gk) * nf + j] = j;
                    const int64_t l = g.dof_ptr[c] + B.conn[k * np + R.face_nodes[j]];
                    for (int d = 0; d < 3; ++d) g.bnode_x.push_back(g.dof_x[size_t(d) * g.ndof + l]);
                }
                continue;
            }
            int other = (c == o) ? nb : o;
            auto it = tri_of[other].find(tkey(f, B.eb[k], B.ea[k]));
            if (it == tri_of[other].end()) {
                err = "unmatched boundary triangle in cell " + std::to_string(c);
                return AFE_E_BAD_MESH;
            }
            int kn = it->second;
            int64_t gkn = g.sub_ptr[other] + kn;
            g.nbr_sub[gk] = int32_t(gkn);
            const CellBuild &Bn = cb[other];
            for (int j = 0; j < nf; ++j) {
                const Key &kj = B.keys[B.conn[k * np + R.face_nodes[j]]];
                int found = -1;
                for (int jj = 0; jj < nf; ++jj)
                    if (Bn.keys[Bn.conn[size_t(kn) * np + R.face_nodes[jj]]] == kj) found = jj;
                if (found < 0) {
                    err = "face nodes do not match across a face";
                    return AFE_E_BAD_MESH;
                }
                g.perm[size_t(gk) * nf + j] = found;
            }
            // triangle geometry is taken from the owner's frame, negated for the neighbour
            if (c != o) {
                const double *To = &cb[o].tri[size_t(kn) * 4];
                double *T = &g.tri[size_t(gk) * 4];
                T[0] = To[0];
                T[1] = -To[1];
                T[2] = -To[2];
                T[3] = -To[3];
            }
        }
    }
    // DOF incidence lists (sub-tet node -> DOF, transposed), ascending
    g.inc_ptr.assign(g.ndof + 1, 0);
    g.finc_ptr.assign(g.ndof + 1, 0);
    for (int64_t k = 0; k < g.nsub; ++k) {
        int64_t d0 = g.dof_ptr[g.sub_cell[k]];
        for (int m = 0; m < np; ++m) g.inc_ptr[d0 + g.conn[k * np + m] + 1]++;
        for (int j = 0; j < nf; ++j) g.finc_ptr[d0 + g.conn[k * np + R.face_nodes[j]] + 1]++;
    }
    for (int64_t l = 0; l < g.ndof; ++l) {
        g.inc_ptr[l + 1] += g.inc_ptr[l];
        g.finc_ptr[l + 1] += g.finc_ptr[l];
    }
    g.inc_idx.resize(g.inc_ptr[g.ndof]);
    g.finc_idx.resize(g.finc_ptr[g.ndof]);
    {
        std::vector<int32_t> fill(g.inc_ptr.begin(), g.inc_ptr.end() - 1), ffill(g.finc_ptr.begin(), g.finc_ptr.end() - 1);
        for (int64_t k = 0; k < g.nsub; ++k) {
            int64_t d0 = g.dof_ptr[g.sub_cell[k]];
            for (int m = 0; m < np; ++m) g.inc_idx[fill[d0 + g.conn[k * np + m]]++] = int32_t(k * np + m);
            for (int j = 0; j < nf; ++j) g.finc_idx[ffill[d0 + g.conn[k * np + R.face_nodes[j]]]++] = int32_t(k * nf + j);
        }
    }
    return AFE_OK;
}

}  // namespace afe
