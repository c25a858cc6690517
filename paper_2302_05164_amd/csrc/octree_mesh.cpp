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

bool oct_build(OctMesh &m, int P, int maxl, const int n0[3], const double L[3], int64_t n_leaves,
               const int32_t *lv, std::string &err)
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
    m.leaf.assign(lv, lv + 4 * n_leaves);
    m.n_cells = n_leaves;
    // validity: aligned, inside, no duplicates or nesting, full cover, 2:1 balance
    long double vol = 0;
    for (int64_t e = 0; e < n_leaves; ++e) {
        const int l = lv[4 * e];
        if (l < 0 || l > maxl) return err = "leaf level out of range", false;
        const int64_t s = 1LL << (maxl - l);
        for (int d = 0; d < 3; ++d) {
            const int64_t o = lv[4 * e + 1 + d];
            if (o < 0 || o % s != 0 || o + s > nf[d]) return err = "leaf not aligned or outside the box", false;
        }
        if (!m.leaf_map.emplace(leaf_key(l, lv[4 * e + 1], lv[4 * e + 2], lv[4 * e + 3]), (int32_t)e).second)
            return err = "duplicate leaf", false;
        vol += (long double)s * s * s;
    }
    if (vol != (long double)nf[0] * nf[1] * nf[2]) return err = "leaves do not cover the box exactly", false;
    for (int64_t e = 0; e < n_leaves; ++e) {
        const int l = lv[4 * e];
        for (int a = 0; a < l; ++a) {
            const int64_t s = 1LL << (maxl - a);
            if (m.leaf_map.count(leaf_key(a, lv[4 * e + 1] / s * s, lv[4 * e + 2] / s * s, lv[4 * e + 3] / s * s)))
                return err = "overlapping leaves", false;
        }
    }
    auto containing = [&](int64_t x, int64_t y, int64_t z) -> int32_t {  // leaf holding finest cell (x,y,z)
        for (int l = maxl; l >= 0; --l) {
            const int64_t s = 1LL << (maxl - l);
            auto it = m.leaf_map.find(leaf_key(l, x / s * s, y / s * s, z / s * s));
            if (it != m.leaf_map.end()) return it->second;
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
                    if (x < 0 || y < 0 || z < 0 || x >= nf[0] || y >= nf[1] || z >= nf[2]) continue;
                    const int32_t nb = containing(x, y, z);
                    if (nb >= 0 && lv[4 * nb] < l - 1) return err = "octree is not 2:1 balanced", false;
                }
    }
    // nodes in order of first appearance
    std::unordered_map<uint64_t, int32_t> node_of;
    node_of.reserve((size_t)n_leaves * 8);
    std::vector<int64_t> nkey;  // 3 per node
    std::vector<int32_t> cnode((size_t)n_leaves * NN);
    for (int64_t e = 0; e < n_leaves; ++e) {
        const int64_t s = 1LL << (maxl - lv[4 * e]);
        for (int a = 0; a < NN; ++a) {
            const int64_t x = lv[4 * e + 1] * P + (a % N1) * s, y = lv[4 * e + 2] * P + ((a / N1) % N1) * s,
                          z = lv[4 * e + 3] * P + (a / (N1 * N1)) * s;
            auto ins = node_of.emplace(lattice_key(x, y, z), (int32_t)(nkey.size() / 3));
            if (ins.second) {
                nkey.push_back(x);
                nkey.push_back(y);
                nkey.push_back(z);
            }
            cnode[(size_t)e * NN + a] = ins.first->second;
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
                        auto it = node_of.find(lattice_key(x[0], x[1], x[2]));
                        if (it == node_of.end() || hanging[it->second]) continue;
                        const int32_t k = it->second;
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
    const int64_t top[3] = {((int64_t)m.n0[0] << m.maxl) * m.P, ((int64_t)m.n0[1] << m.maxl) * m.P,
                            ((int64_t)m.n0[2] << m.maxl) * m.P};
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
        bool powder = false;
        for (int qz = 0; qz <= m.P; ++qz) {
            const double gp = m.P == 1 ? Tables<1>::gp(qz) : Tables<2>::gp(qz);
            if (m.L[2] - (z0 + gp * hz) <= powder_depth) powder = true;
        }
        if (powder) {
            m.cell_hist[e] = (int32_t)m.n_hist_cells++;
            m.hist_z.push_back(z0);
            m.hist_z.push_back(hz);
        }
    }
}

// leaf containing the finest-unit point x (clamped into the box); -1 if none
int32_t oct_locate(const OctMesh &m, const double x[3], double xi[3])
{
    for (int l = m.maxl; l >= 0; --l) {
        const int64_t s = 1LL << (m.maxl - l);
        int64_t o[3];
        for (int d = 0; d < 3; ++d) {
            const int64_t nf = (int64_t)m.n0[d] << m.maxl;
            int64_t c = (int64_t)std::floor(x[d] / s) * s;
            c = std::min(std::max(c, (int64_t)0), nf - s);
            o[d] = c;
        }
        auto it = m.leaf_map.find(leaf_key(l, o[0], o[1], o[2]));
        if (it != m.leaf_map.end()) {
            for (int d = 0; d < 3; ++d) xi[d] = std::min(std::max((x[d] - o[d]) / s, 0.0), 1.0);
            return it->second;
        }
    }
    return -1;
}

}  // namespace pbf
