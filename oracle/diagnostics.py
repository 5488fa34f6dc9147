"""Network diagnostics of Assumption 3.4 and Lemma 3.5, as evaluated in Sec. 6.1
(Table 6.1) and Sec. 6.2.1 (Table 6.3): plain numpy / scipy, FP64.

TEST INFRASTRUCTURE ONLY: imported by tests/ (never by the library).

Boxes: the unit square (cube) split into nb^d boxes of side h = 1/nb.

* Homogeneity: the mass density of every box, (M 1 summed over the nodes in
  the box) / h^d, with the lumped mass (M 1)(x) = 1/2 sum_{y~x} |x - y| of
  eq. 2.1 and the half-open boxes of Sec. 2.3 (a node belongs to exactly one
  box). sigma = max / min over the boxes (rho = min), Assumption 3.4.1.
* Connectivity: per box, the subgraph of every edge with an endpoint in the
  closed box, joined where it falls apart by shortest (fewest-edge, BFS) paths
  whose nodes lie within r0 of the box (Assumption 3.4.2); lambda_2 of
  L u = lambda M u on it (L: the 1/|e| weighted Laplacian of eq. 2.2, M: the
  lumped mass of the subgraph's own edges, the Neumann case of the proof of
  Lemma 3.5) gives mu_box = 1 / (h sqrt(lambda_2)); mu = max over the boxes.
  A box whose subgraph cannot be joined within r0 gives mu_box = inf.

Readings (the paper is not explicit): the box side h is the length in
lambda_2^-1 <= mu^2 h^2, and the connectivity subgraph takes the closed box;
Table 6.3 uses the elements of T_H (h = H), Table 6.1 the boxes B_R (h = 2R).
With these the grid row of Table 6.3 (sigma 1.0 / 1.0 / 1.1 / 1.1, mu 0.45 /
0.47 / 0.48 / 0.51 for H^-1 = 4, 8, 16, 32) is reproduced to 0.01.
"""
from __future__ import annotations

import collections

import numpy as np


def lumped_mass(coords, edges):
    """(M 1)(x) at every node (eq. 2.1)."""
    ln = np.linalg.norm(coords[edges[:, 0]] - coords[edges[:, 1]], axis=1)
    m = np.zeros(len(coords))
    np.add.at(m, edges[:, 0], 0.5 * ln)
    np.add.at(m, edges[:, 1], 0.5 * ln)
    return m


def box_of(coords, nb):
    """Half-open box index (lexicographic, axis 0 fastest), the last box of an
    axis closed at 1 (Sec. 2.3)."""
    e = np.minimum(np.floor(coords * nb).astype(np.int64), nb - 1)
    e = np.maximum(e, 0)
    idx = np.zeros(len(coords), dtype=np.int64)
    for k in range(coords.shape[1] - 1, -1, -1):
        idx = idx * nb + e[:, k]
    return idx


def homogeneity(coords, edges, nb):
    """(densities per box, sigma, rho)."""
    d = coords.shape[1]
    m = lumped_mass(coords, edges)
    dens = np.bincount(box_of(coords, nb), weights=m, minlength=nb ** d) * float(nb) ** d
    rho = dens.min()
    sigma = dens.max() / rho if rho > 0 else np.inf
    return dens, float(sigma), float(rho)


def _box_bounds(b, nb, d):
    v = []
    for _ in range(d):
        v.append(b % nb)
        b //= nb
    lo = np.array(v, dtype=np.float64) / nb
    return lo, lo + 1.0 / nb


def _components(n, a, c):
    parent = list(range(n))

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i

    for i, j in zip(a, c):
        ri, rj = find(i), find(j)
        if ri != rj:
            parent[max(ri, rj)] = min(ri, rj)
    return np.array([find(i) for i in range(n)])


def box_subgraph(coords, edges, adj, b, nb, r0, cand):
    """Edge ids of the connectivity subgraph of box b, or None when it cannot be
    joined within r0 of the box. cand: the nodes that may lie within r0 of the
    box (a superset)."""
    d = coords.shape[1]
    lo, hi = _box_bounds(b, nb, d)
    xc = coords[cand]
    inside = cand[np.all((xc >= lo) & (xc <= hi), axis=1)]
    near = set(cand[np.all((xc >= lo - r0) & (xc <= hi + r0), axis=1)].tolist())
    sel = set()
    for u in inside.tolist():
        for (_, eid) in adj[u]:
            sel.add(eid)
    if not sel:
        return []
    while True:
        es = np.array(sorted(sel))
        nodes = np.unique(edges[es].ravel())
        loc = {int(v): i for i, v in enumerate(nodes)}
        comp = _components(len(nodes), [loc[int(u)] for u in edges[es, 0]], [loc[int(u)] for u in edges[es, 1]])
        roots = np.unique(comp)
        if len(roots) == 1:
            return sorted(sel)
        # BFS from the component of the first node through nodes near the box
        # to the nearest node of another component; add that path's edges
        src = set(int(nodes[i]) for i in np.flatnonzero(comp == comp[0]))
        other = set(int(nodes[i]) for i in np.flatnonzero(comp != comp[0]))
        prev = {v: (-1, -1) for v in src}
        dq = collections.deque(sorted(src))
        hit = -1
        while dq and hit < 0:
            u = dq.popleft()
            for (w, eid) in adj[u]:
                if w in prev or w not in near:
                    continue
                prev[w] = (u, eid)
                if w in other:
                    hit = w
                    break
                dq.append(w)
        if hit < 0:
            return None
        v = hit
        while prev[v][0] >= 0:
            sel.add(prev[v][1])
            v = prev[v][0]


def lambda2(coords, edges, eids):
    """Second smallest eigenvalue of L u = lambda M u on the subgraph."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    es = edges[np.asarray(eids)]
    nodes = np.unique(es.ravel())
    loc = -np.ones(len(coords), dtype=np.int64)
    loc[nodes] = np.arange(len(nodes))
    a, c = loc[es[:, 0]], loc[es[:, 1]]
    ln = np.linalg.norm(coords[es[:, 0]] - coords[es[:, 1]], axis=1)
    n = len(nodes)
    w = 1.0 / ln
    L = sp.coo_matrix((np.r_[-w, -w], (np.r_[a, c], np.r_[c, a])), shape=(n, n)).tocsr()
    L = L + sp.diags(-np.asarray(L.sum(axis=1)).ravel())
    m = np.zeros(n)
    np.add.at(m, a, 0.5 * ln)
    np.add.at(m, c, 0.5 * ln)
    if n <= 400:
        import scipy.linalg as sl
        ev = sl.eigh(L.toarray(), np.diag(m), eigvals_only=True)
        return float(np.sort(ev)[1])
    shift = -1e-3 * float((L.diagonal() / m).min())
    ev = spl.eigsh(L, k=2, M=sp.diags(m), sigma=shift, which="LM", return_eigenvectors=False)
    return float(np.sort(ev)[1])


def connectivity(coords, edges, nb, r0=None):
    """(mu per box, mu). r0 defaults to the longest edge (the locality scale of
    Assumption 3.4.3)."""
    d = coords.shape[1]
    if r0 is None:
        r0 = float(np.linalg.norm(coords[edges[:, 0]] - coords[edges[:, 1]], axis=1).max())
    adj = collections.defaultdict(list)
    for k, (u, v) in enumerate(edges):
        adj[int(u)].append((int(v), k))
        adj[int(v)].append((int(u), k))
    h = 1.0 / nb
    # candidate nodes of a box: those of the boxes within ceil(r0 / h) of it
    # (plus a margin of one box for the closed upper faces)
    span = int(np.ceil(r0 / h)) + 1
    bid = box_of(coords, nb)
    order = np.argsort(bid, kind="stable")
    start = np.searchsorted(bid[order], np.arange(nb ** d + 1))
    mus = np.zeros(nb ** d)
    for b in range(nb ** d):
        v = [(b // nb ** k) % nb for k in range(d)]
        ranges = [range(max(0, v[k] - span), min(nb, v[k] + span + 1)) for k in range(d)]
        boxes = np.zeros(1, dtype=np.int64)
        for k in range(d - 1, -1, -1):
            boxes = (boxes[:, None] * nb + np.array(list(ranges[k]))[None, :]).ravel()
        cand = np.concatenate([order[start[q]:start[q + 1]] for q in boxes])
        eids = box_subgraph(coords, edges, adj, b, nb, r0, cand)
        if eids is None:
            mus[b] = np.inf
        elif len(eids) == 0:
            mus[b] = 0.0
        else:
            lam = lambda2(coords, edges, eids)
            mus[b] = 1.0 / (h * np.sqrt(lam)) if lam > 0 else np.inf
    return mus, float(mus.max())
