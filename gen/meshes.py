"""Mesh-like data-affinity graphs (cfd-style workloads).

The paper's cfd inputs are unstructured meshes in which every particle (cell)
interacts with at most four neighbours (Section 3.3 describes mc2depi's degree
2-4 profile as resembling such meshes).  The meshes here are synthetic stand-ins:

* ``grid2d``: a triangulated W x H lattice, edges right / up / one diagonal.
* ``tet_mesh``: the dual graph of a Kuhn (6-tetrahedra-per-cube) split of an
  a x b x c box of unit cubes with jittered lattice points; one vertex per
  tetrahedron, one edge per interior triangular face.

Conventions shared by both: vertex ids are permuted by a seeded permutation,
every edge is stored with ``u < v`` (in permuted ids), and its geometry is the
unit normal pointing from ``u`` to ``v`` (plus the face area in 3D).
Geometry is returned in float64; callers cast to float32 for the GPU.
"""

from __future__ import annotations

import itertools

import numpy as np


def _rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(tag)])))


_TAG_PERM = 1
_TAG_JITTER = 2


def _orient(edges: np.ndarray, geom_vec: np.ndarray):
    """Store each edge with u < v; flip the direction vector where swapped."""
    u = edges[:, 0].copy()
    v = edges[:, 1].copy()
    swap = u > v
    u[swap], v[swap] = v[swap], u[swap]
    g = geom_vec.copy()
    g[swap] = -g[swap]
    return np.stack([u, v], axis=1), g


def grid2d(W: int = 64, H: int = 64, seed: int = 0, permute: bool = True) -> dict:
    """Triangulated W x H lattice graph.

    Vertex (i, j) (row i, column j) sits at position (x, y) = (j, i) and has
    unpermuted id ``W*i + j``.  Edges: right (i,j)-(i,j+1), up (i,j)-(i+1,j),
    diagonal (i,j)-(i+1,j+1).  Per-edge geometry: the unit normal
    rot_{-90}(p_v - p_u)/|p_v - p_u| = (dy, -dx)/len.
    """
    n = W * H
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    vid = (W * ii + jj).astype(np.int64)
    pos = np.stack([jj.ravel(), ii.ravel()], axis=1).astype(np.float64)  # indexed by vid
    right = np.stack([vid[:, :-1].ravel(), vid[:, 1:].ravel()], axis=1)
    up = np.stack([vid[:-1, :].ravel(), vid[1:, :].ravel()], axis=1)
    diag = np.stack([vid[:-1, :-1].ravel(), vid[1:, 1:].ravel()], axis=1)
    edges = np.concatenate([right, up, diag], axis=0)
    if permute:
        perm = _rng(seed, _TAG_PERM).permutation(n)
    else:
        perm = np.arange(n)
    new_pos = np.empty_like(pos)
    new_pos[perm] = pos
    e = perm[edges]
    d = new_pos[e[:, 1]] - new_pos[e[:, 0]]
    nrm = np.stack([d[:, 1], -d[:, 0]], axis=1)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    e, nrm = _orient(e, nrm)
    order = np.lexsort((e[:, 1], e[:, 0]))
    return {
        "kind": "grid2d",
        "n": n,
        "edges": e[order].astype(np.int32),
        "geom": nrm[order],  # [m, 2] float64: (nx, ny), area 1
        "pos": new_pos,
        "dim": 2,
    }


_PERMS = list(itertools.permutations(range(3)))  # lexicographic; tet t of a cube uses _PERMS[t]


def tet_mesh(a: int, b: int, c: int, seed: int = 0, jitter: float = 0.1, permute: bool = True) -> dict:
    """Dual graph of the Kuhn split of an a x b x c box of unit cubes.

    Cube (i, j, l) holds six tetrahedra; tetrahedron t walks from corner
    (i, j, l) to (i+1, j+1, l+1) stepping along the axes in the order
    ``_PERMS[t]``.  Lattice points are jittered by U(-jitter, jitter) per
    coordinate (jitter is in units of the lattice spacing h = 1).
    Unpermuted cell id: ``6*((i*b + j)*c + l) + t``.

    Returns n = 6abc cells and the m interior faces as edges, with
    geom[e] = (nx, ny, nz, area): the unit normal of the shared face pointing
    from u to v, and the face area.
    """
    rng_j = _rng(seed, _TAG_JITTER)
    P = np.stack(np.meshgrid(np.arange(a + 1), np.arange(b + 1), np.arange(c + 1), indexing="ij"), axis=-1)
    P = P.reshape(-1, 3).astype(np.float64)
    P0 = P.copy()
    if jitter > 0:
        P = P + rng_j.uniform(-jitter, jitter, size=P.shape)

    def pidx(i, j, l):
        return (i * (b + 1) + j) * (c + 1) + l

    ci, cj, cl = np.meshgrid(np.arange(a), np.arange(b), np.arange(c), indexing="ij")
    ci, cj, cl = ci.ravel(), cj.ravel(), cl.ravel()
    ncube = a * b * c
    n = 6 * ncube
    tets = np.empty((ncube, 6, 4), dtype=np.int64)
    for t, pr in enumerate(_PERMS):
        cur = [ci.copy(), cj.copy(), cl.copy()]
        tets[:, t, 0] = pidx(*cur)
        for s in range(3):
            cur[pr[s]] = cur[pr[s]] + 1
            tets[:, t, s + 1] = pidx(*cur)
    tets = tets.reshape(n, 4)

    def vol(X):
        x0, x1, x2, x3 = (X[tets[:, q]] for q in range(4))
        return np.einsum("ij,ij->i", np.cross(x1 - x0, x2 - x0), x3 - x0) / 6.0

    v_ref = vol(P0)
    v_jit = vol(P)
    if not (np.all(np.sign(v_ref) == np.sign(v_jit)) and np.all(np.abs(v_jit) > 1e-3)):
        raise AssertionError("jitter inverted or flattened a tetrahedron")

    # all 4n faces: (sorted point triple, cell, omitted local vertex)
    faces = []
    for omit in range(4):
        keep = [q for q in range(4) if q != omit]
        tri = np.sort(tets[:, keep], axis=1)
        faces.append((tri, np.arange(n), np.full(n, omit)))
    tri = np.concatenate([f[0] for f in faces])
    cell = np.concatenate([f[1] for f in faces])
    omit = np.concatenate([f[2] for f in faces])
    key = (tri[:, 0] << 40) | (tri[:, 1] << 20) | tri[:, 2]
    srt = np.argsort(key, kind="stable")
    key_s = key[srt]
    pair = np.nonzero(key_s[1:] == key_s[:-1])[0]
    fa, fb = srt[pair], srt[pair + 1]
    cu, cv = cell[fa], cell[fb]
    tri_f = tri[fa]
    opp_u = tets[cu, omit[fa]]

    x0, x1, x2 = P[tri_f[:, 0]], P[tri_f[:, 1]], P[tri_f[:, 2]]
    A = 0.5 * np.cross(x1 - x0, x2 - x0)
    # orient outward from cu: away from its vertex opposite the face
    s = np.einsum("ij,ij->i", A, x0 - P[opp_u])
    A[s < 0] *= -1.0

    if permute:
        perm = _rng(seed, _TAG_PERM).permutation(n)
    else:
        perm = np.arange(n)
    e = np.stack([perm[cu], perm[cv]], axis=1)
    e, A = _orient(e, A)
    order = np.lexsort((e[:, 1], e[:, 0]))
    e, A = e[order], A[order]
    area = np.linalg.norm(A, axis=1)
    geom = np.concatenate([A / area[:, None], area[:, None]], axis=1)
    centroid = np.empty((n, 3))
    centroid[perm] = P[tets].mean(axis=1)
    return {
        "kind": "tet_mesh",
        "n": n,
        "edges": e.astype(np.int32),
        "geom": geom,  # [m, 4] float64
        "centroid": centroid,
        "dim": 3,
        "shape": (a, b, c),
    }


def default_order(edges: np.ndarray) -> np.ndarray:
    """Index order an application iterating its own cells emits: sort by (u, v)."""
    return np.lexsort((edges[:, 1], edges[:, 0]))


def bfs_subgraph(mesh: dict, n_keep: int = 1000, root: int = 0) -> dict:
    """Induced subgraph on the first ``n_keep`` vertices in BFS order from ``root``.

    Neighbours are visited in ascending id; the kept vertices are renumbered in
    BFS order; edges are re-stored with u < v, flipping the normal where the
    renumbering swaps the endpoints.
    """
    n = mesh["n"]
    e = mesh["edges"].astype(np.int64)
    adj = [[] for _ in range(n)]
    for u, v in e:
        adj[u].append(v)
        adj[v].append(u)
    seen = np.full(n, -1, dtype=np.int64)
    queue = [root]
    seen[root] = 0
    head = 0
    cnt = 1
    while head < len(queue) and cnt < n_keep:
        w = queue[head]
        head += 1
        for x in sorted(adj[w]):
            if seen[x] < 0 and cnt < n_keep:
                seen[x] = cnt
                cnt += 1
                queue.append(x)
    keep = (seen[e[:, 0]] >= 0) & (seen[e[:, 1]] >= 0)
    ne = np.stack([seen[e[keep, 0]], seen[e[keep, 1]]], axis=1)
    g = mesh["geom"][keep].copy()
    d = mesh["dim"]
    vec = g[:, :d]
    ne, vec = _orient(ne, vec)
    g[:, :d] = vec
    order = np.lexsort((ne[:, 1], ne[:, 0]))
    out = dict(mesh)
    out.update(n=cnt, edges=ne[order].astype(np.int32), geom=g[order], kind=mesh["kind"] + "_bfs")
    out.pop("centroid", None)
    out.pop("pos", None)
    return out
