// Host construction of octree meshes with hanging nodes: node lattice, hanging
// constraints, degrees of freedom and the tables the device kernels read.
//
// Leaves are given as (level, ix, iy, iz), the origin in units of the finest
// cell (coarse cell / 2^max_level).  Nodes live on the lattice of step
// finest/P.  Continuity across a level change (Section 4.2: the gather G_e
// includes the constraints of hanging nodes) is imposed by making every node
// that lies on a face of a coarser leaf, at a position that is not one of
// that leaf's nodes, a hanging node: its value is the coarse leaf's
// interpolant there, a product of 1D Lagrange weights of degree P at the
// quarter points of the face ((3/8, 3/4, -1/8) for P = 2, (1/2, 1/2) for P = 1).
// In a 2:1 balanced tree these are all the non-conforming nodes, and they sit
// at odd half-node positions of the coarse face.  Constraints whose masters
// hang themselves are expanded down to regular nodes, the degrees of freedom.
//
// Device tables: per cell and local node the dof or the hanging id (SoA),
// the expanded constraints (CSR), and per dof the list of (cell, local node,
// weight) contributions in a fixed order (the transposed gather), so that the
// scatter is a deterministic gather on the node side.  The lumped mass of a
// dof is the sum of its weighted element row sums.
#include <algorithm>
#include <cmath>
#include <functional>
#include <unordered_map>

#include "pbf_internal.h"

namespace pbf {
namespace {

inline uint64_t lattice_key(int64_t x, int64_t y, int64_t z)
{
    return (uint64_t)x | ((uint64_t)y << 21) | ((uint64_t)z << 42);
}

// leaf origins are below 2^20 finest cells per direction, levels below 16
inline uint64_t leaf_key(int l, int64_t x, int64_t y, int64_t z)
{
    return (uint64_t)x | ((uint64_t)y << 20) | ((uint64_t)z << 40) | ((uint64_t)l << 60);
}

// 1D Lagrange basis of degree P on equispaced nodes at x = t / (2P)
double lag1(int P, int b, int t)
{
    const double x = double(t) / (2.0 * P);
    if (P == 1) return b == 0 ? 1.0 - x : x;
    if (b == 0) return 2.0 * (x - 0.5) * (x - 1.0);
    if (b == 1) return 4.0 * x * (1.0 - x);
    return 2.0 * x * (x - 0.5);
}

}  // namespace

// Leaves of the octree refined around a window of the scan path (the octree
// workload: every cell within `radius` of the beam path between arc lengths
// s_lo and s_hi reaches max_level).  The path is sampled at points at most
// half a finest cell apart; a level-l cell is split when its box comes closer
// than R_{l+1} to a sampled point, with R_max = radius and R_l = R_{l+1} + (the
// diagonal of a level-l cell): the graded radii keep the tree 2:1 balanced
// across faces, edges and vertices.  Output in Morton order of the origins.
#pragma STDC FP_CONTRACT OFF
bool oct_path_leaves(const int n0[3], const double L[3], int maxl, double radius, const double *tracks,
                     int n_tracks, double s_lo, double s_hi, std::vector<int32_t> &out, std::string &err)
{
    if (maxl < 0 || maxl > 15) return err = "max_level must be in [0, 15]", false;
    for (int d = 0; d < 3; ++d)
        if (n0[d] < 1 || !(L[d] > 0)) return err = "coarse cells and box lengths must be positive", false;
    if (!(radius >= 0) || !std::isfinite(s_lo) || !std::isfinite(s_hi)) return err = "bad radius or window", false;
    double h0[3], unit[3];
    for (int d = 0; d < 3; ++d) {
        h0[d] = L[d] / n0[d];
        unit[d] = h0[d] / (double)(1LL << maxl);
    }
    std::vector<double> R(maxl + 1);
    R[maxl] = radius;
    for (int l = maxl - 1; l >= 0; --l) {
        double a[3], q = 0.0;
        for (int d = 0; d < 3; ++d) a[d] = h0[d] / (double)(1LL << l);
        q = a[0] * a[0];
        q = q + a[1] * a[1];
        q = q + a[2] * a[2];
        R[l] = R[l + 1] + std::sqrt(q);
    }
    // sampled path points
    const double spacing = 0.5 * std::min(unit[0], std::min(unit[1], unit[2]));
    std::vector<double> pts;
    double s0 = 0.0;
    for (int k = 0; k < n_tracks; ++k) {
        const double *tr = tracks + 8 * k;
        double dv[3], q;
        for (int d = 0; d < 3; ++d) dv[d] = tr[3 + d] - tr[d];
        q = dv[0] * dv[0];
        q = q + dv[1] * dv[1];
        q = q + dv[2] * dv[2];
        const double length = std::sqrt(q);
        const double lo = std::max(s_lo, s0), hi = std::min(s_hi, s0 + length);
        if (hi >= lo && length > 0) {
            const int64_t n = std::max<int64_t>(2, (int64_t)std::ceil((hi - lo) / spacing) + 1);
            const double step = (hi - lo) / (double)(n - 1);
            for (int64_t i = 0; i < n; ++i) {
                double v = (double)i * step;
                v = v + lo;
                if (i == n - 1) v = hi;
                const double u = (v - s0) / length;
                for (int d = 0; d < 3; ++d) {
                    double w = u * dv[d];
                    pts.push_back(tr[d] + w);
                }
            }
        }
        s0 += length;
    }
    const int64_t np = (int64_t)pts.size() / 3;
    // bins of the points in x and y (the distance test only visits nearby bins)
    const double bin = std::max(R[0], 4.0 * spacing);
    double pmin[2] = {0, 0};
    int64_t nb[2] = {1, 1};
    if (np > 0) {
        double pmax[2];
        for (int d = 0; d < 2; ++d) pmin[d] = pmax[d] = pts[d];
        for (int64_t i = 0; i < np; ++i)
            for (int d = 0; d < 2; ++d) {
                pmin[d] = std::min(pmin[d], pts[3 * i + d]);
                pmax[d] = std::max(pmax[d], pts[3 * i + d]);
            }
        for (int d = 0; d < 2; ++d) nb[d] = (int64_t)((pmax[d] - pmin[d]) / bin) + 1;
    }
    std::vector<std::vector<int64_t>> bins((size_t)(nb[0] * nb[1]));
    for (int64_t i = 0; i < np; ++i) {
        const int64_t bx = std::min<int64_t>(nb[0] - 1, (int64_t)((pts[3 * i] - pmin[0]) / bin));
        const int64_t by = std::min<int64_t>(nb[1] - 1, (int64_t)((pts[3 * i + 1] - pmin[1]) / bin));
        bins[(size_t)(bx + nb[0] * by)].push_back(i);
    }
    // level by level: cells as origins in finest units
    std::vector<int64_t> g, next;
    for (int64_t ix = 0; ix < n0[0]; ++ix)
        for (int64_t iy = 0; iy < n0[1]; ++iy)
            for (int64_t iz = 0; iz < n0[2]; ++iz) {
                g.push_back(ix << maxl);
                g.push_back(iy << maxl);
                g.push_back(iz << maxl);
            }
    std::vector<int64_t> leaves;  // (level, x, y, z)
    for (int l = 0; l <= maxl; ++l) {
        const int64_t size = 1LL << (maxl - l), half = size / 2;
        const double r2 = l < maxl ? R[l + 1] * R[l + 1] : 0.0;
        next.clear();
        for (size_t c = 0; c < g.size() / 3; ++c) {
            bool split = false;
            if (l < maxl && np > 0) {
                double lo[3], hi[3];
                for (int d = 0; d < 3; ++d) {
                    lo[d] = (double)g[3 * c + d] * unit[d];
                    hi[d] = (double)(g[3 * c + d] + size) * unit[d];
                }
                const double reach = R[l + 1];
                const int64_t bx0 = std::max<int64_t>(0, (int64_t)std::floor((lo[0] - reach - pmin[0]) / bin));
                const int64_t bx1 = std::min<int64_t>(nb[0] - 1, (int64_t)std::floor((hi[0] + reach - pmin[0]) / bin));
                const int64_t by0 = std::max<int64_t>(0, (int64_t)std::floor((lo[1] - reach - pmin[1]) / bin));
                const int64_t by1 = std::min<int64_t>(nb[1] - 1, (int64_t)std::floor((hi[1] + reach - pmin[1]) / bin));
                for (int64_t by = by0; by <= by1 && !split; ++by)
                    for (int64_t bx = bx0; bx <= bx1 && !split; ++bx)
                        for (int64_t i : bins[(size_t)(bx + nb[0] * by)]) {
                            double d2 = 0.0;
                            for (int d = 0; d < 3; ++d) {
                                const double q = pts[3 * i + d];
                                const double e = std::max(std::max(lo[d] - q, 0.0), q - hi[d]);
                                const double ee = e * e;
                                d2 = d == 0 ? ee : d2 + ee;
                            }
                            if (d2 < r2) {
                                split = true;
                                break;
                            }
                        }
            }
            if (!split) {
                leaves.push_back(l);
                for (int d = 0; d < 3; ++d) leaves.push_back(g[3 * c + d]);
            } else {
                for (int k = 0; k < 2; ++k)
                    for (int j = 0; j < 2; ++j)
                        for (int i = 0; i < 2; ++i) {
                            next.push_back(g[3 * c] + i * half);
                            next.push_back(g[3 * c + 1] + j * half);
                            next.push_back(g[3 * c + 2] + k * half);
                        }
            }
        }
        g.swap(next);
    }
    const size_t n = leaves.size() / 4;
    std::vector<std::pair<uint64_t, size_t>> key(n);
    for (size_t e = 0; e < n; ++e) {
        uint64_t k = 0;
        const uint64_t x = (uint64_t)leaves[4 * e + 1], y = (uint64_t)leaves[4 * e + 2], z = (uint64_t)leaves[4 * e + 3];
        for (int b = 0; b < 21; ++b)
            k |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2);
        key[e] = {k, e};
    }
    std::stable_sort(key.begin(), key.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    out.resize(4 * n);
    for (size_t e = 0; e < n; ++e)
        for (int d = 0; d < 4; ++d) out[4 * e + d] = (int32_t)leaves[4 * key[e].second + d];
    return true;
}
#pragma STDC FP_CONTRACT ON

bool oct_build(OctMesh &m, int P, int maxl, const int n0[3], const double L[3], int64_t n_leaves,
               const int32_t *lv, std::string &err, int64_t top)
{
    m = OctMesh{};
    m.P = P;
    m.maxl = maxl;
    for (int d = 0; d < 3; ++d) {
        m.n0[d] = n0[d];
        m.L[d] = L[d];
        m.unit[d] = L[d] / n0[d] / (double)(1LL << maxl);
    }
    const int N1 = P + 1, NN = N1 * N1 * N1;
    if (maxl < 0 || maxl > 15) return err = "max_level must be in [0, 15]", false;
    const int64_t nf[3] = {(int64_t)n0[0] << maxl, (int64_t)n0[1] << maxl, (int64_t)n0[2] << maxl};
    for (int d = 0; d < 3; ++d)
        if (nf[d] * P >= (1LL << 21) || nf[d] >= (1LL << 20))
            return err = "octree too fine for the node lattice", false;
    if (n_leaves < 1 || n_leaves * NN >= (1LL << 31)) return err = "number of leaves out of range", false;
    if (top < 0) top = nf[2];
    if (top < 1 || top > nf[2]) return err = "active top outside the box", false;
    m.top = top;
    const int64_t ext[3] = {nf[0], nf[1], top};  // the active part
    m.leaf.assign(lv, lv + 4 * n_leaves);
    m.n_cells = n_leaves;
    m.leaf_map.reserve((size_t)n_leaves);
    // validity: aligned, inside, no duplicates or nesting, full cover, 2:1 balance
    long double vol = 0;
    for (int64_t e = 0; e < n_leaves; ++e) {
        const int l = lv[4 * e];
        if (l < 0 || l > maxl) return err = "leaf level out of range", false;
        const int64_t s = 1LL << (maxl - l);
        for (int d = 0; d < 3; ++d) {
            const int64_t o = lv[4 * e + 1 + d];
            if (o < 0 || o % s != 0 || o + s > ext[d]) return err = "leaf not aligned or outside the active part", false;
        }
        if (!m.leaf_map.insert(leaf_key(l, lv[4 * e + 1], lv[4 * e + 2], lv[4 * e + 3]), (int32_t)e).second)
            return err = "duplicate leaf", false;
        vol += (long double)s * s * s;
    }
    if (vol != (long double)ext[0] * ext[1] * ext[2]) return err = "leaves do not cover the active part exactly", false;
    for (int64_t e = 0; e < n_leaves; ++e) {
        const int l = lv[4 * e];
        for (int a = 0; a < l; ++a) {
            const int64_t s = 1LL << (maxl - a);
            if (m.leaf_map.find(leaf_key(a, lv[4 * e + 1] / s * s, lv[4 * e + 2] / s * s, lv[4 * e + 3] / s * s)) >= 0)
                return err = "overlapping leaves", false;
        }
    }
    auto containing = [&](int64_t x, int64_t y, int64_t z) -> int32_t {  // leaf holding finest cell (x,y,z)
        for (int l = maxl; l >= 0; --l) {
            const int64_t s = 1LL << (maxl - l);
            const int32_t f = m.leaf_map.find(leaf_key(l, x / s * s, y / s * s, z / s * s));
            if (f >= 0) return f;
        }
        return -1;
    };
    for (int64_t e = 0; e < n_leaves; ++e) {
        const int l = lv[4 * e];
        if (l < 2) continue;
        const int64_t s = 1LL << (maxl - l);
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int64_t x = lv[4 * e + 1] + dx * s, y = lv[4 * e + 2] + dy * s, z = lv[4 * e + 3] + dz * s;
                    if (x < 0 || y < 0 || z < 0 || x >= ext[0] || y >= ext[1] || z >= ext[2]) continue;
                    const int32_t nb = containing(x, y, z);
                    if (nb >= 0 && lv[4 * nb] < l - 1) return err = "octree is not 2:1 balanced", false;
                }
    }
    // nodes in order of first appearance
    FlatMap node_of;
    node_of.reserve((size_t)n_leaves * 9);
    std::vector<int64_t> nkey;  // 3 per node
    std::vector<int32_t> cnode((size_t)n_leaves * NN);
    for (int64_t e = 0; e < n_leaves; ++e) {
        const int64_t s = 1LL << (maxl - lv[4 * e]);
        for (int a = 0; a < NN; ++a) {
            const int64_t x = lv[4 * e + 1] * P + (a % N1) * s, y = lv[4 * e + 2] * P + ((a / N1) % N1) * s,
                          z = lv[4 * e + 3] * P + (a / (N1 * N1)) * s;
            const auto ins = node_of.insert(lattice_key(x, y, z), (int32_t)(nkey.size() / 3));
            if (ins.second) {
                nkey.push_back(x);
                nkey.push_back(y);
                nkey.push_back(z);
            }
            cnode[(size_t)e * NN + a] = ins.first;
        }
    }
    const int64_t n_nodes = (int64_t)nkey.size() / 3;
    // hanging nodes: odd half-node positions on the faces of coarser leaves
    std::vector<std::vector<std::pair<int32_t, double>>> direct(n_nodes);  // masters (nodes) and weights
    std::vector<char> hanging(n_nodes, 0);
    for (int64_t e = 0; e < n_leaves; ++e) {
        const int l = lv[4 * e];
        if (l >= maxl) continue;
        const int64_t s = 1LL << (maxl - l), half = s / 2;
        const int64_t o[3] = {lv[4 * e + 1] * P, lv[4 * e + 2] * P, lv[4 * e + 3] * P};
        for (int nd = 0; nd < 3; ++nd)
            for (int side = 0; side < 2; ++side) {
                const int t1d = (nd + 1) % 3, t2d = (nd + 2) % 3;
                for (int t2 = 0; t2 <= 2 * P; ++t2)
                    for (int t1 = 0; t1 <= 2 * P; ++t1) {
                        if (!(t1 & 1) && !(t2 & 1)) continue;
                        int64_t x[3];
                        x[nd] = o[nd] + side * P * s;
                        x[t1d] = o[t1d] + t1 * half;
                        x[t2d] = o[t2d] + t2 * half;
                        const int32_t k = node_of.find(lattice_key(x[0], x[1], x[2]));
                        if (k < 0 || hanging[k]) continue;
                        hanging[k] = 1;
                        for (int b2 = 0; b2 <= P; ++b2)
                            for (int b1 = 0; b1 <= P; ++b1) {
                                const double w = lag1(P, b1, t1) * lag1(P, b2, t2);
                                if (w == 0.0) continue;
                                int bl[3];
                                bl[nd] = side * P;
                                bl[t1d] = b1;
                                bl[t2d] = b2;
                                const int a = bl[0] + N1 * (bl[1] + N1 * bl[2]);
                                direct[k].emplace_back(cnode[(size_t)e * NN + a], w);
                            }
                    }
            }
    }
    // dofs: regular nodes in order
    std::vector<int32_t> dof(n_nodes, -1), hid(n_nodes, -1);
    for (int64_t k = 0; k < n_nodes; ++k) {
        if (hanging[k]) hid[k] = (int32_t)m.n_hanging++;
        else dof[k] = (int32_t)m.n_dofs++;
    }
    // closure of hanging nodes down to dofs, sorted by dof
    std::vector<std::vector<std::pair<int32_t, double>>> clos(n_nodes);
    std::vector<char> done(n_nodes, 0);
    std::function<void(int32_t)> expand = [&](int32_t k) {
        if (done[k]) return;
        std::vector<std::pair<int32_t, double>> out;
        for (auto &mw : direct[k]) {
            if (!hanging[mw.first]) {
                out.emplace_back(dof[mw.first], mw.second);
            } else {
                expand(mw.first);
                for (auto &dw : clos[mw.first]) out.emplace_back(dw.first, mw.second * dw.second);
            }
        }
        std::sort(out.begin(), out.end(), [](auto &x, auto &y) { return x.first < y.first; });
        std::vector<std::pair<int32_t, double>> merged;
        for (auto &dw : out) {
            if (!merged.empty() && merged.back().first == dw.first) merged.back().second += dw.second;
            else merged.push_back(dw);
        }
        clos[k] = merged;
        done[k] = 1;
    };
    m.hstart.assign(m.n_hanging + 1, 0);
    for (int64_t k = 0; k < n_nodes; ++k)
        if (hanging[k]) {
            expand((int32_t)k);
            m.hstart[hid[k] + 1] = (int32_t)clos[k].size();
        }
    for (int64_t h = 0; h < m.n_hanging; ++h) m.hstart[h + 1] += m.hstart[h];
    m.hdof.resize(m.hstart[m.n_hanging]);
    m.hw.resize(m.hstart[m.n_hanging]);
    for (int64_t k = 0; k < n_nodes; ++k)
        if (hanging[k])
            for (size_t j = 0; j < clos[k].size(); ++j) {
                m.hdof[m.hstart[hid[k]] + j] = clos[k][j].first;
                m.hw[m.hstart[hid[k]] + j] = clos[k][j].second;
            }
    // per-cell local -> dof / hanging id (SoA)
    m.cidx.resize((size_t)NN * n_leaves);
    for (int64_t e = 0; e < n_leaves; ++e)
        for (int a = 0; a < NN; ++a) {
            const int32_t k = cnode[(size_t)e * NN + a];
            m.cidx[(size_t)a * n_leaves + e] = hanging[k] ? -1 - hid[k] : dof[k];
        }
    // transposed gather: per dof the (slot, weight) entries in (cell, node) order
    m.nstart.assign(m.n_dofs + 1, 0);
    auto for_entries = [&](auto &&fn) {
        for (int64_t e = 0; e < n_leaves; ++e)
            for (int a = 0; a < NN; ++a) {
                const int32_t k = cnode[(size_t)e * NN + a];
                const int64_t slot = (int64_t)a * n_leaves + e;
                if (!hanging[k]) fn(dof[k], slot, 1.0, e, a);
                else
                    for (auto &dw : clos[k]) fn(dw.first, slot, dw.second, e, a);
            }
    };
    for_entries([&](int32_t d, int64_t, double, int64_t, int) { ++m.nstart[d + 1]; });
    for (int64_t i = 0; i < m.n_dofs; ++i) m.nstart[i + 1] += m.nstart[i];
    if ((int64_t)m.nstart[m.n_dofs] >= (1LL << 31)) return err = "too many scatter entries", false;
    m.nslot.resize(m.nstart[m.n_dofs]);
    m.nw.resize(m.nstart[m.n_dofs]);
    m.mass.assign(m.n_dofs, 0.0);
    std::vector<int32_t> fill(m.nstart.begin(), m.nstart.end() - 1);
    const double m1[2][3] = {{0.5, 0.5, 0.0}, {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0}};
    for_entries([&](int32_t d, int64_t slot, double w, int64_t e, int a) {
        m.nslot[fill[d]] = (int32_t)slot;
        m.nw[fill[d]] = w;
        ++fill[d];
        const double s = (double)(1LL << (maxl - lv[4 * e]));
        const double me = m1[P - 1][a % N1] * s * m.unit[0] * m1[P - 1][(a / N1) % N1] * s * m.unit[1] *
                          m1[P - 1][a / (N1 * N1)] * s * m.unit[2];
        m.mass[d] += w * me;
    });
    // the weights (constraint products of Lagrange values at dyadic points) are
    // normally exact in FP32: then the node pass reads them in half the bytes
    m.nw_f32 = true;
    for (double w : m.nw) m.nw_f32 = m.nw_f32 && (double)(float)w == w;
    m.nwf.clear();
    if (m.nw_f32) m.nwf.assign(m.nw.begin(), m.nw.end());
    // dof coordinates and lattice keys
    m.dof_key.resize(3 * m.n_dofs);
    m.coords.resize(3 * m.n_dofs);
    for (int64_t k = 0; k < n_nodes; ++k)
        if (!hanging[k])
            for (int d = 0; d < 3; ++d) {
                m.dof_key[3 * dof[k] + d] = nkey[3 * k + d];
                m.coords[3 * dof[k] + d] = nkey[3 * k + d] * m.unit[d] / P;
            }
    return true;
}

// Dirichlet flags (face mask) and the history cells (leaves with a Gauss point
// at most powder_depth below the top face)
void oct_finish(OctMesh &m, unsigned dmask, double powder_depth)
{
    const int64_t top[3] = {((int64_t)m.n0[0] << m.maxl) * m.P, ((int64_t)m.n0[1] << m.maxl) * m.P, m.top * m.P};
    const double ztop = (double)m.top * m.unit[2];
    m.dflag.assign(m.n_dofs, 0);
    for (int64_t i = 0; i < m.n_dofs; ++i)
        for (int d = 0; d < 3; ++d) {
            if ((dmask & (1u << (2 * d))) && m.dof_key[3 * i + d] == 0) m.dflag[i] = 1;
            if ((dmask & (2u << (2 * d))) && m.dof_key[3 * i + d] == top[d]) m.dflag[i] = 1;
        }
    m.cell_hist.assign(m.n_cells, -1);
    m.hist_z.clear();
    m.n_hist_cells = 0;
    for (int64_t e = 0; e < m.n_cells; ++e) {
        const double s = (double)(1LL << (m.maxl - m.leaf[4 * e]));
        const double z0 = m.leaf[4 * e + 3] * m.unit[2], hz = s * m.unit[2];
        bool powder = m.growing && powder_depth >= 0.0;  // growing builds: every deposited leaf
        for (int qz = 0; qz <= m.P; ++qz) {
            const double gp = m.P == 1 ? Tables<1>::gp(qz) : Tables<2>::gp(qz);
            if (ztop - (z0 + gp * hz) <= powder_depth) powder = true;
        }
        if (powder) {
            m.cell_hist[e] = (int32_t)m.n_hist_cells++;
            m.hist_z.push_back(z0);
            m.hist_z.push_back(hz);
        }
    }
}

int32_t oct_locate(const OctMesh &m, const double x[3], double xi[3])
{
    for (int l = m.maxl; l >= 0; --l) {
        const int64_t s = 1LL << (m.maxl - l);
        int64_t o[3];
        for (int d = 0; d < 3; ++d) {
            const int64_t nf = d == 2 ? m.top : (int64_t)m.n0[d] << m.maxl;  // the active part
            int64_t c = (int64_t)std::floor(x[d] / s) * s;
            c = std::min(std::max(c, (int64_t)0), nf - s);
            o[d] = c;
        }
        const int32_t f = m.leaf_map.find(leaf_key(l, o[0], o[1], o[2]));
        if (f >= 0) {
            for (int d = 0; d < 3; ++d) xi[d] = std::min(std::max((x[d] - o[d]) / s, 0.0), 1.0);
            return f;
        }
    }
    return -1;
}

// Leaves of the active part of a growing build after the activation of the
// layer [m.top, new_top) (Section 4.1; new_top == m.top: the refinement of the
// current top layer alone).  Cells of the current layer and those whose
// distance to it is at most d_haz (finest units) are refined to the finest
// level; an octet of sibling leaves farther than d_haz below the current layer
// is replaced by its parent if rc_min (the smallest consolidated fraction of
// each leaf) exceeds r_coarsen in all eight (one level per activation); the
// new layer is added at the finest level; then leaves two or more levels
// coarser than a leaf they touch (face, edge or vertex) are split until the
// tree is 2:1 balanced.  Output in Morton order of the origins.
bool oct_layer_leaves(const OctMesh &m, const std::vector<double> &rc_min, int64_t new_top, int64_t d_haz,
                      double r_coarsen, std::vector<int32_t> &out, std::string &err)
{
    const int maxl = m.maxl;
    const int64_t nf[3] = {(int64_t)m.n0[0] << maxl, (int64_t)m.n0[1] << maxl, (int64_t)m.n0[2] << maxl};
    if (new_top < m.top || new_top > nf[2]) return err = "new top below the current top or outside the box", false;
    if ((int64_t)rc_min.size() != m.n_cells) return err = "one consolidated fraction per leaf expected", false;
    const int64_t layer_bottom = new_top - std::max<int64_t>(1, new_top - m.top);
    auto size = [&](int64_t l) { return (int64_t)1 << (maxl - l); };
    // octets of sibling leaves: sort leaves of level >= 1 by parent
    std::vector<std::pair<uint64_t, int64_t>> byp;
    for (int64_t e = 0; e < m.n_cells; ++e) {
        const int64_t l = m.leaf[4 * e];
        if (l == 0) continue;
        const int64_t ps = size(l - 1);
        byp.push_back({leaf_key((int)(l - 1), m.leaf[4 * e + 1] / ps * ps, m.leaf[4 * e + 2] / ps * ps,
                                m.leaf[4 * e + 3] / ps * ps), e});
    }
    std::sort(byp.begin(), byp.end());
    FlatMap coarsen;  // parent key -> 0 (not yet emitted) / 1 (emitted)
    for (size_t i = 0; i < byp.size();) {
        size_t j = i;
        while (j < byp.size() && byp[j].first == byp[i].first) ++j;
        if (j - i == 8) {
            const int64_t e = byp[i].second, l = m.leaf[4 * e], ps = size(l - 1);
            const int64_t pz = m.leaf[4 * e + 3] / ps * ps;
            bool ok = layer_bottom - (pz + ps) > d_haz;
            for (size_t k = i; k < j && ok; ++k) ok = rc_min[byp[k].second] > r_coarsen;
            if (ok) coarsen.insert(byp[i].first, 0);
        }
        i = j;
    }
    std::vector<int64_t> cur;  // (level, x, y, z)
    auto push = [&](int64_t l, int64_t x, int64_t y, int64_t z) {
        cur.push_back(l);
        cur.push_back(x);
        cur.push_back(y);
        cur.push_back(z);
    };
    std::function<void(int64_t, int64_t, int64_t, int64_t)> refine_full = [&](int64_t l, int64_t x, int64_t y,
                                                                                int64_t z) {
        if (l == maxl) return push(l, x, y, z);
        const int64_t h = size(l) / 2;
        for (int k = 0; k < 2; ++k)
            for (int j = 0; j < 2; ++j)
                for (int i = 0; i < 2; ++i) refine_full(l + 1, x + i * h, y + j * h, z + k * h);
    };
    FlatMap emitted;
    for (int64_t e = 0; e < m.n_cells; ++e) {
        const int64_t l = m.leaf[4 * e], x = m.leaf[4 * e + 1], y = m.leaf[4 * e + 2], z = m.leaf[4 * e + 3];
        if (l > 0) {
            const int64_t ps = size(l - 1);
            const uint64_t pk = leaf_key((int)(l - 1), x / ps * ps, y / ps * ps, z / ps * ps);
            if (coarsen.find(pk) >= 0) {
                if (emitted.insert(pk, 1).second) push(l - 1, x / ps * ps, y / ps * ps, z / ps * ps);
                continue;
            }
        }
        if (z + size(l) > layer_bottom - d_haz && l < maxl) refine_full(l, x, y, z);
        else push(l, x, y, z);
    }
    for (int64_t z = m.top; z < new_top; ++z)
        for (int64_t y = 0; y < nf[1]; ++y)
            for (int64_t x = 0; x < nf[0]; ++x) push(maxl, x, y, z);
    // 2:1 balance by refinement
    const int64_t ext[3] = {nf[0], nf[1], new_top};
    for (;;) {
        const size_t n = cur.size() / 4;
        FlatMap at;
        at.reserve(n);
        for (size_t e = 0; e < n; ++e) at.insert(leaf_key((int)cur[4 * e], cur[4 * e + 1], cur[4 * e + 2], cur[4 * e + 3]), (int32_t)e);
        std::vector<char> split(n, 0);
        bool any = false;
        for (size_t e = 0; e < n; ++e) {
            const int64_t l = cur[4 * e];
            if (l < 2) continue;
            const int64_t s = size(l);
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (!dx && !dy && !dz) continue;
                        const int64_t p[3] = {cur[4 * e + 1] + (dx < 0 ? -1 : dx * s), cur[4 * e + 2] + (dy < 0 ? -1 : dy * s),
                                              cur[4 * e + 3] + (dz < 0 ? -1 : dz * s)};
                        bool in = true;
                        for (int d = 0; d < 3; ++d) in = in && p[d] >= 0 && p[d] < ext[d];
                        if (!in) continue;
                        for (int64_t a = 0; a <= l - 2; ++a) {  // a leaf at least two levels coarser holding p
                            const int64_t sa = size(a);
                            const int32_t f = at.find(leaf_key((int)a, p[0] / sa * sa, p[1] / sa * sa, p[2] / sa * sa));
                            if (f >= 0) {
                                split[f] = 1;
                                any = true;
                                break;
                            }
                        }
                    }
        }
        if (!any) break;
        std::vector<int64_t> nxt;
        for (size_t e = 0; e < n; ++e) {
            if (!split[e]) {
                for (int d = 0; d < 4; ++d) nxt.push_back(cur[4 * e + d]);
                continue;
            }
            const int64_t l = cur[4 * e], h = size(l) / 2;
            for (int k = 0; k < 2; ++k)
                for (int j = 0; j < 2; ++j)
                    for (int i = 0; i < 2; ++i) {
                        nxt.push_back(l + 1);
                        nxt.push_back(cur[4 * e + 1] + i * h);
                        nxt.push_back(cur[4 * e + 2] + j * h);
                        nxt.push_back(cur[4 * e + 3] + k * h);
                    }
        }
        cur.swap(nxt);
    }
    const size_t n = cur.size() / 4;
    std::vector<std::pair<uint64_t, size_t>> key(n);
    for (size_t e = 0; e < n; ++e) {
        uint64_t k = 0;
        const uint64_t x = (uint64_t)cur[4 * e + 1], y = (uint64_t)cur[4 * e + 2], z = (uint64_t)cur[4 * e + 3];
        for (int b = 0; b < 21; ++b)
            k |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2);
        key[e] = {k, e};
    }
    std::stable_sort(key.begin(), key.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    out.resize(4 * n);
    for (size_t e = 0; e < n; ++e)
        for (int d = 0; d < 4; ++d) out[4 * e + d] = (int32_t)cur[4 * key[e].second + d];
    return true;
}

}  // namespace pbf
