"""Seeded synthetic inputs: trees, fields and kernel tables.

This module produces inputs only. It holds none of the integration
arithmetic, so both the test oracle and the device path may consume what
it generates without sharing any of the method's code.

A tree is returned as ``(parent, weight)``:

* ``parent`` -- int64[N]; ``parent[v] == -1`` marks a root, several roots
  make a forest (no interaction between its trees);
* ``weight`` -- int32[N]; ``weight[v] >= 1`` is the integer length of the
  edge ``(v, parent[v])`` and is ignored (set to 0) at roots.

Integer weights are lattice lengths: the paper integrates real-weighted
trees only after quantising every edge to a positive integer number of
lattice units (appendix on distance quantisation, ``q_e = max(1,
round(w_e / Delta))``).

Generators cover the workloads the library is measured on and the
deterministic and random tree families of the paper's synthetic benchmark
appendix (table of deterministic constructions; random recursive,
random-MST topology and preferential-attachment families).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "edges_to_parent", "relabel", "forest",
    "path", "star", "balanced_kary", "caterpillar", "caterpillar_hanging_paths",
    "comb", "broom", "double_broom", "spider",
    "random_recursive", "random_mst_topology", "preferential_attachment",
    "binary_random_recursive", "grid_mst", "sphere_knn_mst",
    "patch_grid_tree", "attention_features", "attention_payload",
    "paper_families",
    "topo_mask_table",
    "uniform_weights", "normal_field", "dirichlet_field",
    "exp_table", "inv_sq_table", "inv_table", "expsum_table", "ones_table",
    "workload",
]


# ---------------------------------------------------------------- helpers --

def edges_to_parent(n, u, v, w=None, root=0):
    """Orient an undirected tree (edge lists ``u``, ``v``, weights ``w``)
    away from ``root`` and return ``(parent, weight)``. Several connected
    components give a forest rooted at the smallest vertex of each."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    if w is None:
        w = np.ones(len(u), dtype=np.int64)
    w = np.asarray(w, dtype=np.int64)
    deg = np.bincount(np.concatenate([u, v]), minlength=n)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=off[1:])
    nbr = np.empty(2 * len(u), dtype=np.int64)
    nw = np.empty(2 * len(u), dtype=np.int64)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    ww = np.concatenate([w, w])
    order = np.argsort(src, kind="stable")
    nbr[:] = dst[order]
    nw[:] = ww[order]
    parent = np.full(n, -2, dtype=np.int64)
    weight = np.zeros(n, dtype=np.int32)
    roots = [root] + [r for r in range(n) if r != root]
    for r in roots:
        if parent[r] != -2:
            continue
        parent[r] = -1
        stack = [r]
        while stack:
            x = stack.pop()
            for k in range(off[x], off[x + 1]):
                y = nbr[k]
                if parent[y] == -2:
                    parent[y] = x
                    weight[y] = nw[k]
                    stack.append(y)
    return parent, weight


def relabel(parent, weight, perm):
    """Return the same tree with vertex ``v`` renamed ``perm[v]``."""
    parent = np.asarray(parent)
    perm = np.asarray(perm, dtype=np.int64)
    n = len(parent)
    p2 = np.full(n, -1, dtype=np.int64)
    w2 = np.zeros(n, dtype=np.int32)
    nz = parent >= 0
    p2[perm[nz]] = perm[parent[nz]]
    w2[perm] = weight
    w2[p2 < 0] = 0
    return p2, w2


def forest(trees):
    """Concatenate trees ``[(parent, weight), ...]`` into one forest;
    returns ``(parent, weight, offsets)`` with tree ``i`` occupying vertices
    ``offsets[i]:offsets[i+1]``."""
    ps, ws, offs = [], [], [0]
    for p, w in trees:
        p = np.asarray(p, dtype=np.int64)
        ps.append(np.where(p >= 0, p + offs[-1], -1))
        ws.append(np.asarray(w, dtype=np.int32))
        offs.append(offs[-1] + len(p))
    return (np.concatenate(ps), np.concatenate(ws),
            np.asarray(offs, dtype=np.int64))


def uniform_weights(parent, lo, hi, rng):
    """Integer weights uniform in ``{lo..hi}`` on every non-root vertex."""
    w = rng.integers(lo, hi + 1, size=len(parent)).astype(np.int32)
    w[np.asarray(parent) < 0] = 0
    return w


def _unit(parent):
    w = np.ones(len(parent), dtype=np.int32)
    w[np.asarray(parent) < 0] = 0
    return w


# ----------------------------------------- deterministic paper families --

def path(n):
    p = np.arange(-1, n - 1, dtype=np.int64)
    return p, _unit(p)


def star(n):
    p = np.zeros(n, dtype=np.int64)
    p[0] = -1
    return p, _unit(p)


def balanced_kary(k, depth):
    """Complete k-ary tree of the given depth (edges root->leaf)."""
    n = (k ** (depth + 1) - 1) // (k - 1)
    p = np.empty(n, dtype=np.int64)
    p[0] = -1
    idx = np.arange(1, n)
    p[1:] = (idx - 1) // k
    return p, _unit(p)


def caterpillar(spine, leaves_per_vertex=3):
    """Spine ``0..spine-1`` (a path) with ``leaves_per_vertex`` leaves per
    spine vertex; leaf ``j`` of spine vertex ``t`` is
    ``spine + t*leaves_per_vertex + j``."""
    n = spine * (1 + leaves_per_vertex)
    p = np.empty(n, dtype=np.int64)
    p[:spine] = np.arange(-1, spine - 1)
    p[spine:] = np.repeat(np.arange(spine), leaves_per_vertex)
    return p, _unit(p)


def caterpillar_hanging_paths(ell):
    """Spine of ``ell`` vertices with an ``ell``-edge path hanging from
    every spine vertex; ``N = ell + ell**2``."""
    n = ell + ell * ell
    p = np.empty(n, dtype=np.int64)
    p[:ell] = np.arange(-1, ell - 1)
    for t in range(ell):
        base = ell + t * ell
        p[base] = t
        p[base + 1: base + ell] = np.arange(base, base + ell - 1)
    return p, _unit(p)


def comb(spine):
    return caterpillar(spine, 2)


def broom(ell):
    """Handle of ``ell`` vertices with ``ell/2`` leaves at one end."""
    h = ell
    k = ell // 2
    p = np.empty(h + k, dtype=np.int64)
    p[:h] = np.arange(-1, h - 1)
    p[h:] = h - 1
    return p, _unit(p)


def double_broom(ell):
    """Handle of ``ell`` vertices with ``ell/4`` leaves at each end."""
    h = ell
    k = ell // 4
    p = np.empty(h + 2 * k, dtype=np.int64)
    p[:h] = np.arange(-1, h - 1)
    p[h:h + k] = 0
    p[h + k:] = h - 1
    return p, _unit(p)


def spider(arms, arm_len):
    """Hub 0 with ``arms`` paths of ``arm_len`` edges."""
    n = 1 + arms * arm_len
    p = np.empty(n, dtype=np.int64)
    p[0] = -1
    for a in range(arms):
        base = 1 + a * arm_len
        p[base] = 0
        p[base + 1: base + arm_len] = np.arange(base, base + arm_len - 1)
    return p, _unit(p)


# ------------------------------------------------------- random families --

def random_recursive(n, rng):
    """Vertex ``i`` attaches to a uniform parent in ``[0, i)``."""
    p = np.empty(n, dtype=np.int64)
    p[0] = -1
    if n > 1:
        p[1:] = rng.integers(0, np.arange(1, n, dtype=np.int64))
    return p, _unit(p)


def binary_random_recursive(n, rng):
    """Vertex ``i`` attaches to a uniform vertex of ``[0, i)`` that still
    has fewer than two children."""
    p = np.empty(n, dtype=np.int64)
    p[0] = -1
    avail = np.empty(n, dtype=np.int64)
    nchild = np.zeros(n, dtype=np.int8)
    pos = np.full(n, -1, dtype=np.int64)
    avail[0] = 0
    pos[0] = 0
    cnt = 1
    u = rng.random(n)
    for i in range(1, n):
        j = int(u[i] * cnt)
        if j >= cnt:
            j = cnt - 1
        par = int(avail[j])
        p[i] = par
        nchild[par] += 1
        if nchild[par] == 2:
            last = int(avail[cnt - 1])
            avail[j] = last
            pos[last] = j
            cnt -= 1
        avail[cnt] = i
        pos[i] = cnt
        cnt += 1
    return p, _unit(p)


def _mst_edges(n, u, v, key):
    """Minimum spanning forest of the graph with (distinct) edge keys."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import minimum_spanning_tree
    g = sp.coo_matrix((key, (u, v)), shape=(n, n)).tocsr()
    t = minimum_spanning_tree(g).tocoo()
    return t.row.astype(np.int64), t.col.astype(np.int64)


def random_mst_topology(n, rng):
    """Kruskal MST of the complete graph with i.i.d. uniform [0,1) edge
    weights; the weights are discarded (unit edges)."""
    iu, ju = np.triu_indices(n, 1)
    key = rng.random(len(iu)) + 1e-12
    r, c = _mst_edges(n, iu, ju, key)
    return edges_to_parent(n, r, c)


def preferential_attachment(n, rng):
    """Sampling-list construction: a new vertex picks a uniform entry of
    the list, then the parent and itself are appended."""
    p = np.empty(n, dtype=np.int64)
    p[0] = -1
    lst = np.empty(2 * n, dtype=np.int64)
    lst[0] = 0
    m = 1
    u = rng.random(n)
    for i in range(1, n):
        j = min(int(u[i] * m), m - 1)
        par = lst[j]
        p[i] = par
        lst[m] = par
        lst[m + 1] = i
        m += 2
    return p, _unit(p)


def grid_mst(side, wmax, rng):
    """Minimum spanning tree of a ``side x side`` 4-neighbour grid with
    integer edge weights uniform in ``{1..wmax}``; ties are broken by edge
    index (row-major, right edge before down edge), i.e. Kruskal with a
    stable sort. The MST keeps its weights."""
    s = side
    n = s * s
    idx = np.arange(n).reshape(s, s)
    # interleave right/down per vertex in row-major order
    right = np.full((s, s), -1, dtype=np.int64)
    right[:, :-1] = idx[:, 1:]
    down = np.full((s, s), -1, dtype=np.int64)
    down[:-1, :] = idx[1:, :]
    src = np.repeat(idx.ravel(), 2)
    dst = np.stack([right.ravel(), down.ravel()], axis=1).ravel()
    keep = dst >= 0
    us = src[keep]
    vs = dst[keep]
    m = len(us)
    w = rng.integers(1, wmax + 1, size=m)
    key = w.astype(np.float64) + (np.arange(m, dtype=np.float64) + 1) / (m + 2)
    r, c = _mst_edges(n, us, vs, key)
    # recover the integer weight of every chosen edge
    lut = {}
    for a, b, ww in zip(us.tolist(), vs.tolist(), w.tolist()):
        lut[(a, b)] = ww
        lut[(b, a)] = ww
    tw = np.array([lut[(a, b)] for a, b in zip(r.tolist(), c.tolist())],
                  dtype=np.int64)
    return edges_to_parent(n, r, c, tw)


# ------------------------------------------- synthetic family sweep --

def paper_families(seed=0):
    """The fifteen families of the paper's synthetic benchmark at the
    largest size of each sweep (appendix table of deterministic
    constructions; table "synthetic-largest"), unit weights:
    ``[(name, parent, weight), ...]``. The three random families use
    ``default_rng(seed)``, N = 800."""
    rng = np.random.default_rng(seed)
    fam = [
        ("path", *path(800)),
        ("balanced_binary", *balanced_kary(2, 9)),
        ("complete_3ary", *balanced_kary(3, 6)),
        ("caterpillar", *caterpillar(400, 3)),
        ("caterpillar_hanging_paths", *caterpillar_hanging_paths(32)),
        ("comb", *comb(400)),
        ("broom", *broom(640)),
        ("double_broom", *double_broom(320)),
        ("uniform_spider", *spider(30, 25)),
        ("short_arm_spider", *spider(400, 2)),
        ("long_arm_spider", *spider(8, 500)),
        ("star", *star(800)),
        ("random_recursive", *random_recursive(800, rng)),
        ("random_mst_topology", *random_mst_topology(800, rng)),
        ("preferential_attachment", *preferential_attachment(800, rng)),
    ]
    return fam


# ------------------------------------------ patch-grid spanning trees --

def _hilbert_order(s):
    """Grid cells ``(row, col)`` of an ``s x s`` grid (``s`` a power of
    two) in Hilbert-curve order, as row-major ids."""
    n = s * s
    t = np.arange(n, dtype=np.int64)
    x = np.zeros(n, dtype=np.int64)
    y = np.zeros(n, dtype=np.int64)
    q = 1
    while q < s:
        rx = 1 & (t // 2)
        ry = 1 & (t ^ rx)
        flip = ry == 0
        swap_x = np.where(flip & (rx == 1), q - 1 - x, x)
        swap_y = np.where(flip & (rx == 1), q - 1 - y, y)
        x, y = np.where(flip, swap_y, swap_x), np.where(flip, swap_x, swap_y)
        x = x + q * rx
        y = y + q * ry
        t = t // 4
        q *= 2
    return y * s + x


def patch_grid_tree(kind, side, rng=None):
    """Spanning tree of the unit-weight ``side x side`` 4-neighbour patch
    grid, vertices numbered row-major (vertex ``i*side + j`` is patch
    ``(i, j)``), as in the tree sweep of the paper's vision-transformer
    appendix (subsection "Tree families"):

    ``serpentine``  row-major boustrophedon Hamiltonian path;
    ``hilbert``     Hilbert-curve Hamiltonian path (``side`` a power of 2);
    ``comb``        spine on row 0, a full-height tooth below every column;
    ``fishbone``    spine on the central row ``side // 2``, ribs up and down
                    every column;
    ``random``      Kruskal spanning tree with i.i.d. uniform edge keys
                    (``rng`` required).
    """
    s = int(side)
    n = s * s
    idx = np.arange(n, dtype=np.int64).reshape(s, s)
    if kind in ("serpentine", "hilbert"):
        if kind == "serpentine":
            rows = idx.copy()
            rows[1::2] = rows[1::2, ::-1]
            order = rows.ravel()
        else:
            if s & (s - 1):
                raise ValueError("hilbert needs a power-of-two side")
            order = _hilbert_order(s)
        p = np.empty(n, dtype=np.int64)
        p[order[0]] = -1
        p[order[1:]] = order[:-1]
        return p, _unit(p)
    if kind == "comb":
        p = np.empty((s, s), dtype=np.int64)
        p[0, 0] = -1
        p[0, 1:] = idx[0, :-1]
        p[1:, :] = idx[:-1, :]
        p = p.ravel()
        return p, _unit(p)
    if kind == "fishbone":
        c = s // 2
        p = np.empty((s, s), dtype=np.int64)
        p[c, 0] = -1
        p[c, 1:] = idx[c, :-1]
        p[:c, :] = idx[1:c + 1, :]
        p[c + 1:, :] = idx[c:-1, :]
        p = p.ravel()
        return p, _unit(p)
    if kind == "random":
        if rng is None:
            raise ValueError("random needs an rng")
        right_u = idx[:, :-1].ravel()
        right_v = idx[:, 1:].ravel()
        down_u = idx[:-1, :].ravel()
        down_v = idx[1:, :].ravel()
        us = np.concatenate([right_u, down_u])
        vs = np.concatenate([right_v, down_v])
        key = rng.random(len(us)) + 1e-12
        r, c = _mst_edges(n, us, vs, key)
        return edges_to_parent(n, r, c)
    raise KeyError(kind)


def attention_features(n, r, dh, rng):
    """Per-token positive random features ``phi[n x r]`` (log-normal,
    unit mean) and values ``v[n x dh]`` ~ N(0,1), both FP32."""
    phi = np.exp(0.5 * rng.standard_normal((n, r)) - 0.125).astype(np.float32)
    v = rng.standard_normal((n, dh)).astype(np.float32)
    return phi, v


def attention_payload(phi, v):
    """Stacked masked-linear-attention payload of the paper's reduction
    (appendix "Masked linear attention as tree-field integration"):
    ``x_j = [vec(phi_j v_j^T) | phi_j]`` with ``C = r*(dh+1)`` channels,
    channel ``a*dh + b`` holding ``phi_j[a] v_j[b]`` and channel
    ``r*dh + a`` holding ``phi_j[a]``."""
    phi = np.asarray(phi)
    v = np.asarray(v)
    n, r = phi.shape
    outer = (phi[:, :, None] * v[:, None, :]).reshape(n, -1)
    return np.concatenate([outer, phi], axis=1)


def topo_mask_table(length, u, v, w):
    """Topological mask ``f(k) = exp(u k^2 + v k + w)`` on the lattice."""
    k = np.arange(length, dtype=np.float64)
    return np.exp(u * k * k + v * k + w)


def sphere_knn_mst(n, k, bins_per_unit, rng):
    """``n`` points uniform on the unit sphere, symmetrised k-NN graph,
    Euclidean MST (components joined by their shortest connecting edge),
    lengths quantised as ``max(1, round(len * bins_per_unit))``."""
    from scipy.spatial import cKDTree
    x = rng.standard_normal((n, 3))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    tree = cKDTree(x)
    dist, nb = tree.query(x, k=k + 1)
    u = np.repeat(np.arange(n), k)
    v = nb[:, 1:].ravel()
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    pairs = np.unique(a * n + b)
    a = pairs // n
    b = pairs % n
    length = np.linalg.norm(x[a] - x[b], axis=1)
    r, c = _mst_edges(n, a, b, length)
    # join components of the spanning forest (rare for k=8)
    par, _ = edges_to_parent(n, r, c)
    roots = np.flatnonzero(par < 0)
    if len(roots) > 1:
        comp = _components(par)
        extra_r, extra_c = [], []
        while True:
            labels = np.unique(comp)
            if len(labels) == 1:
                break
            lab0 = comp[0]
            ins = np.flatnonzero(comp == lab0)
            out = np.flatnonzero(comp != lab0)
            t2 = cKDTree(x[out])
            dd, jj = t2.query(x[ins], k=1)
            i0 = int(np.argmin(dd))
            p0, q0 = int(ins[i0]), int(out[jj[i0]])
            extra_r.append(p0)
            extra_c.append(q0)
            comp[comp == comp[q0]] = lab0
        r = np.concatenate([r, np.array(extra_r, dtype=np.int64)])
        c = np.concatenate([c, np.array(extra_c, dtype=np.int64)])
    length = np.linalg.norm(x[r] - x[c], axis=1)
    q = np.maximum(1, np.rint(length * bins_per_unit)).astype(np.int64)
    return edges_to_parent(n, r, c, q)


def _components(parent):
    n = len(parent)
    comp = np.arange(n)
    order = _topo(parent)
    for v in order:
        if parent[v] >= 0:
            comp[v] = comp[parent[v]]
    return comp


def _topo(parent):
    """Vertices in an order where every parent precedes its children."""
    n = len(parent)
    children = [[] for _ in range(n)]
    roots = []
    for v in range(n):
        if parent[v] < 0:
            roots.append(v)
        else:
            children[parent[v]].append(v)
    out = []
    stack = roots[::-1]
    while stack:
        x = stack.pop()
        out.append(x)
        stack.extend(children[x])
    return out


# --------------------------------------------------- fields and kernels --

def normal_field(n, d, rng, dtype=np.float64):
    return rng.standard_normal((n, d)).astype(dtype)


def dirichlet_field(n, rng, dtype=np.float64):
    return rng.dirichlet(np.ones(n)).astype(dtype)


def exp_table(length, lam):
    """``f(k) = exp(-lam * k)`` on the integer lattice."""
    k = np.arange(length, dtype=np.float64)
    return np.exp(-lam * k)


def inv_sq_table(length):
    """``f(k) = 1 / (1 + k)^2``."""
    k = np.arange(length, dtype=np.float64)
    return 1.0 / (1.0 + k) ** 2


def inv_table(length):
    """``f(k) = 1 / (1 + k)`` (the paper's synthetic-benchmark kernel)."""
    k = np.arange(length, dtype=np.float64)
    return 1.0 / (1.0 + k)


def expsum_table(length, a, b):
    """``f(k) = sum_j a_j * exp(-b_j * k)``."""
    k = np.arange(length, dtype=np.float64)[:, None]
    return (np.asarray(a)[None, :] * np.exp(-k * np.asarray(b)[None, :])).sum(1)


def ones_table(length):
    return np.ones(length, dtype=np.float64)


# ------------------------------------------------------------ workloads --

def workload(name, seed=None, **kw):
    """Named workloads with the shapes of the measured configurations.

    ``small``   random recursive tree, N=2000, weights U{1..4}, F[N x 4]
                FP64 ~ N(0,1), f = exp(-0.1 d).
    ``rrt100k`` random recursive tree, N=100000, weights U{1..8}, F[N x 16]
                FP32 ~ N(0,1), kernels exp(-0.05 d) and 1/(1+d)^2.
    ``grid512`` 512 grid-MST trees (side U{14..64}), weights U{1..16},
                F[n x 64] FP32, f = sum_{k<8} a_k exp(-b_k d).
    ``sphere50k`` sphere kNN MST, N=50000, k=8, lattice 1/64,
                f = exp(-d/3.2) in lattice units, Dirichlet(1) marginals.
    ``cater2m`` / ``binary2m`` N=2e6 caterpillar / binary random recursive
                tree, weights U{1..8}, F[N x 32] FP32, f = exp(-0.01 d).
    ``attn``    masked linear attention on a ``side x side`` patch grid
                (``tree`` = serpentine, hilbert, comb, fishbone or random;
                default serpentine, side 256), unit weights, features
                phi[N x 64] and values v[N x 64] (payload C = 4160 channels,
                built by ``attention_payload``), mask
                f = exp(u d^2 + v d + w) with u = -1e-5, v = -0.01, w = 0.5.

    Returns a dict with ``parent``, ``weight``, ``F`` and workload metadata;
    kernel tables are built by the caller once the required table length is
    known (``kernels`` lists them as ``(name, callable(length))``).
    """
    if name == "small":
        rng = np.random.default_rng(1 if seed is None else seed)
        n = kw.get("n", 2000)
        p, _ = random_recursive(n, rng)
        w = uniform_weights(p, 1, 4, rng)
        F = normal_field(n, kw.get("d", 4), rng)
        return dict(parent=p, weight=w, F=F, dtype="f64",
                    kernels=[("exp0.1", lambda L: exp_table(L, 0.1))])
    if name == "rrt100k":
        rng = np.random.default_rng(2 if seed is None else seed)
        n = kw.get("n", 100_000)
        p, _ = random_recursive(n, rng)
        w = uniform_weights(p, 1, 8, rng)
        F = normal_field(n, kw.get("d", 16), rng, np.float32)
        return dict(parent=p, weight=w, F=F, dtype="f32",
                    kernels=[("exp0.05", lambda L: exp_table(L, 0.05)),
                             ("invsq", inv_sq_table)])
    if name == "grid512":
        rng = np.random.default_rng(3 if seed is None else seed)
        ntrees = kw.get("trees", 512)
        smin, smax = kw.get("side", (14, 64))
        sides = rng.integers(smin, smax + 1, size=ntrees)
        trees = [grid_mst(int(s), 16, rng) for s in sides]
        p, w, offs = forest(trees)
        d = kw.get("d", 64)
        F = normal_field(len(p), d, rng, np.float32)
        a = rng.standard_normal(8)
        b = rng.uniform(0.01, 0.5, size=8)
        return dict(parent=p, weight=w, F=F, offsets=offs, a=a, b=b,
                    dtype="f32",
                    kernels=[("expsum8", lambda L: expsum_table(L, a, b))])
    if name == "sphere50k":
        rng = np.random.default_rng(4 if seed is None else seed)
        n = kw.get("n", 50_000)
        p, w = sphere_knn_mst(n, 8, 64, rng)
        a = dirichlet_field(n, rng)
        b = dirichlet_field(n, rng)
        return dict(parent=p, weight=w, a=a, b=b, dtype="f32",
                    kernels=[("exp/3.2", lambda L: exp_table(L, 1 / 3.2))])
    if name in ("cater2m", "binary2m"):
        rng = np.random.default_rng(5 if seed is None else seed)
        n = kw.get("n", 2_000_000)
        if name == "cater2m":
            p, _ = caterpillar(n // 4, 3)
        else:
            p, _ = binary_random_recursive(n, rng)
        w = uniform_weights(p, 1, 8, rng)
        F = normal_field(len(p), kw.get("d", 32), rng, np.float32)
        return dict(parent=p, weight=w, F=F, dtype="f32",
                    kernels=[("exp0.01", lambda L: exp_table(L, 0.01))])
    if name == "attn":
        rng = np.random.default_rng(6 if seed is None else seed)
        side = kw.get("side", 256)
        kind = kw.get("tree", "serpentine")
        p, w = patch_grid_tree(kind, side, rng)
        r = kw.get("r", 64)
        dh = kw.get("dh", 64)
        phi, v = attention_features(len(p), r, dh, rng)
        mask = (-1e-5, -0.01, 0.5)
        return dict(parent=p, weight=w, phi=phi, v=v, dtype="f32", mask=mask,
                    d=r * (dh + 1), tree=kind, side=side,
                    kernels=[("topo", lambda L: topo_mask_table(L, *mask))])
    raise KeyError(name)
