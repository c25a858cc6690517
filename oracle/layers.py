"""Per-layer mesh adaptation of a growing build (Section 4.1, "Mesh adaptivity
and layer activation"), written out plainly for the tests.

TEST INFRASTRUCTURE ONLY: slow (quadratic in the number of leaves), shares no
code with the GPU library.

Leaves are rows (level, ix, iy, iz), origins in units of the finest cell; the
coarse cells have size 2^max_level; the finest cell is as tall as a powder
layer (eq. coarse_fine_relation: h_coarse = 2^n_refine h_powder), so layer
boundaries are cell faces.  The active part is z < top (finest units); cells
above it are inactive and carry no dofs (they are not listed).

When a new layer [old_top, new_top) is activated:
  - all cells of the current (top-most) layer are refined to the finest level;
  - cells whose distance to the current layer is at most d_HAZ stay refined
    (are refined to the finest level if they are not);
  - an octet of sibling leaves farther than d_HAZ from the current layer is
    replaced by its parent if the consolidated fraction exceeds r_coarsen at
    every quadrature point of all eight (one level per activation);
  - the mesh is then made 2:1 balanced across faces, edges and vertices by
    refinement (refinement wins over coarsening).
"""
import numpy as np


def _size(level, max_level):
    return 1 << (max_level - level)


def morton_order(leaves):
    lv = np.asarray(leaves, dtype=np.int64).reshape(-1, 4)
    key = np.zeros(len(lv), dtype=np.int64)
    for b in range(21):
        key |= ((lv[:, 1] >> b) & 1) << (3 * b) | ((lv[:, 2] >> b) & 1) << (3 * b + 1) | \
               ((lv[:, 3] >> b) & 1) << (3 * b + 2)
    return lv[np.argsort(key, kind="stable")]


def split(leaf, max_level):
    l, x, y, z = leaf
    h = _size(l, max_level) // 2
    return [(l + 1, x + i * h, y + j * h, z + k * h) for k in (0, 1) for j in (0, 1) for i in (0, 1)]


def balance(leaves, max_level):
    """Refine until every two leaves that touch (share a face, an edge or a
    vertex) differ by at most one level: the coarser of a pair two or more
    levels apart is split, repeatedly."""
    cur = [tuple(map(int, r)) for r in leaves]
    while True:
        a = np.array(cur, dtype=np.int64)
        lo = a[:, 1:]
        s = np.array([_size(l, max_level) for l in a[:, 0]], dtype=np.int64)
        hi = lo + s[:, None]
        # touching: closed boxes intersect (interiors are disjoint in a valid mesh)
        touch = np.ones((len(a), len(a)), dtype=bool)
        for d in range(3):
            touch &= (lo[:, None, d] <= hi[None, :, d]) & (lo[None, :, d] <= hi[:, None, d])
        lev = a[:, 0]
        bad = touch & (lev[None, :] - lev[:, None] >= 2)  # row leaf is >= 2 levels coarser than a neighbour
        to_split = np.nonzero(bad.any(axis=1))[0]
        if len(to_split) == 0:
            return morton_order(a)
        keep = np.ones(len(cur), dtype=bool)
        keep[to_split] = False
        nxt = [cur[i] for i in range(len(cur)) if keep[i]]
        for i in to_split:
            nxt.extend(split(cur[i], max_level))
        cur = nxt


def initial_leaves(n0, max_level, top, d_haz):
    """The start of a build: coarse cells below z = top (a multiple of the coarse
    size), the top layer [top - 1, top) and the cells within d_haz of it at the
    finest level, balanced."""
    sc = 1 << max_level
    assert top % sc == 0
    coarse = [(0, i * sc, j * sc, k * sc) for k in range(top // sc) for j in range(n0[1]) for i in range(n0[0])]
    return adapt(coarse, None, max_level, n0, top, top, d_haz, 0.9)


def adapt(leaves, rc_min, max_level, n0, old_top, new_top, d_haz, r_coarsen):
    """Leaves of the active part after activating the layer [old_top, new_top)
    (finest units; old_top == new_top: only the refinement of the current top
    layer [top - 1, top)).  rc_min[e]: the smallest consolidated fraction over
    the quadrature points of leaf e (None: 1 everywhere).  d_haz in finest
    units."""
    lv = [tuple(map(int, r)) for r in leaves]
    rc = np.ones(len(lv)) if rc_min is None else np.asarray(rc_min, dtype=np.float64)
    layer_bottom = new_top - max(1, new_top - old_top)
    zmax = lambda r: r[3] + _size(r[0], max_level)
    # octets of sibling leaves farther than d_haz below the current layer
    parent_of = {}
    for e, r in enumerate(lv):
        if r[0] == 0:
            continue
        ps = _size(r[0] - 1, max_level)
        parent_of.setdefault((r[0] - 1, r[1] // ps * ps, r[2] // ps * ps, r[3] // ps * ps), []).append(e)
    coarsen = set()
    for par, kids in parent_of.items():
        if len(kids) != 8:
            continue
        if layer_bottom - zmax(par) <= d_haz:  # not farther than d_HAZ from the current layer
            continue
        if min(rc[k] for k in kids) > r_coarsen:
            coarsen.add(par)
    out = []
    done = set()
    for e, r in enumerate(lv):
        if r[0] > 0:
            ps = _size(r[0] - 1, max_level)
            par = (r[0] - 1, r[1] // ps * ps, r[2] // ps * ps, r[3] // ps * ps)
            if par in coarsen:
                if par not in done:
                    out.append(par)
                    done.add(par)
                continue
        if zmax(r) > layer_bottom - d_haz and r[0] < max_level:  # current layer or HAZ: finest level
            stack = [r]
            while stack:
                c = stack.pop()
                if c[0] == max_level:
                    out.append(c)
                else:
                    stack.extend(split(c, max_level))
        else:
            out.append(r)
    # the new layer at the finest level
    nfx, nfy = n0[0] << max_level, n0[1] << max_level
    for z in range(old_top, new_top):
        for y in range(nfy):
            for x in range(nfx):
                out.append((max_level, x, y, z))
    return balance(out, max_level)


def rc_min_per_leaf(rc_leafmajor, n_leaves, nq):
    return np.asarray(rc_leafmajor, dtype=np.float64).reshape(n_leaves, nq).min(axis=1)
