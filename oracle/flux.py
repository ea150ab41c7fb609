"""The cfd-style pairwise interaction, forward and adjoint, in FP64.

The paper's cfd task computes the interaction of two adjacent particles from
their density, momentum and energy and applies it to both (Section 1, Figure 1;
Section 3.1).  It prints no formula, so this project fixes one (FLUX5): an
Euler normal flux with central averaging plus a constant-coefficient
dissipation term, a textbook finite-volume form that needs only add, multiply
and divide.

State q = (rho, m1, m2, m3, E); edge geometry: unit normal n from u to v
(2D: n3 = 0) and face area a (2D: a = 1); gamma = 1.4, sigma = 1.0.
  s(q)   = (m . n) / rho
  p(q)   = (gamma - 1) (E - |m|^2 / (2 rho))
  f(q)   = (rho s, m1 s + p n1, m2 s + p n2, m3 s + p n3, (E + p) s)
  F_e    = (f(q_u) + f(q_v)) / 2 - sigma (q_v - q_u) / 2
  r[u_e] += a_e F_e ;  r[v_e] -= a_e F_e ;  q_new = q + dt r

Everything here evaluates on unpacked (original-id) inputs with no partition
involved, straight from the definition.
"""

from __future__ import annotations

import numpy as np

GAMMA = 1.4
SIGMA = 1.0


def split_geom(geom: np.ndarray):
    """(unit normal [m,3], area [m]) from 2 (nx, ny) or 4 (nx, ny, nz, a) floats."""
    geom = np.asarray(geom, dtype=np.float64)
    m = len(geom)
    if geom.ndim == 1:
        geom = geom.reshape(m, -1)
    g = geom.shape[1]
    if g == 2:
        return np.concatenate([geom, np.zeros((m, 1))], axis=1), np.ones(m)
    if g == 4:
        return geom[:, :3].copy(), geom[:, 3].copy()
    raise ValueError("geometry must have 2 or 4 components per edge")


def euler_flux(q: np.ndarray, n: np.ndarray) -> np.ndarray:
    q = np.asarray(q, dtype=np.float64)
    rho, mom, E = q[:, 0], q[:, 1:4], q[:, 4]
    s = np.einsum("ij,ij->i", mom, n) / rho
    p = (GAMMA - 1.0) * (E - 0.5 * np.einsum("ij,ij->i", mom, mom) / rho)
    f = np.empty_like(q)
    f[:, 0] = rho * s
    f[:, 1:4] = mom * s[:, None] + p[:, None] * n
    f[:, 4] = (E + p) * s
    return f


def edge_flux(qu: np.ndarray, qv: np.ndarray, n: np.ndarray) -> np.ndarray:
    return 0.5 * (euler_flux(qu, n) + euler_flux(qv, n)) - 0.5 * SIGMA * (qv - qu)


def forward(n_vertices: int, edges: np.ndarray, geom: np.ndarray, q: np.ndarray, dt: float | None = None):
    """r[n][5] (and q_new if dt is given) from the definition."""
    edges = np.asarray(edges, dtype=np.int64)
    q = np.asarray(q, dtype=np.float64)
    nrm, area = split_geom(geom)
    u, v = edges[:, 0], edges[:, 1]
    F = edge_flux(q[u], q[v], nrm) * area[:, None]
    r = np.zeros((n_vertices, 5))
    np.add.at(r, u, F)
    np.add.at(r, v, -F)
    if dt is None:
        return r
    return r, q + dt * r


def forward_abs(n_vertices: int, edges: np.ndarray, geom: np.ndarray, q: np.ndarray, dt: float | None = None):
    """Absolute-value evaluation of ``forward``: the same expression on |inputs|
    with every subtraction turned into an addition.  It bounds the magnitudes
    that rounding acts on and floors the elementwise tolerance."""
    edges = np.asarray(edges, dtype=np.int64)
    q = np.abs(np.asarray(q, dtype=np.float64))
    nrm, area = split_geom(geom)
    nrm, area = np.abs(nrm), np.abs(area)

    def fabs(qq):
        rho, mom, E = qq[:, 0], qq[:, 1:4], qq[:, 4]
        s = np.einsum("ij,ij->i", mom, nrm) / rho
        p = (GAMMA - 1.0) * (E + 0.5 * np.einsum("ij,ij->i", mom, mom) / rho)
        f = np.empty_like(qq)
        f[:, 0] = rho * s
        f[:, 1:4] = mom * s[:, None] + p[:, None] * nrm
        f[:, 4] = (E + p) * s
        return f

    u, v = edges[:, 0], edges[:, 1]
    F = (0.5 * (fabs(q[u]) + fabs(q[v])) + 0.5 * SIGMA * (q[v] + q[u])) * area[:, None]
    r = np.zeros((n_vertices, 5))
    np.add.at(r, u, F)
    np.add.at(r, v, F)
    if dt is None:
        return r
    return r, q + abs(dt) * r


def euler_jacobian(q: np.ndarray, n: np.ndarray, absolute: bool = False) -> np.ndarray:
    """J[e, k, j] = d f_k / d q_j at state q[e] and normal n[e] (hand-derived).

    With s = m.n/rho and p as above:
      ds/drho = -s/rho, ds/dm_i = n_i/rho;
      dp/drho = (gamma-1)|m|^2/(2 rho^2), dp/dm_i = -(gamma-1) m_i/rho, dp/dE = gamma-1.
    ``absolute=True`` gives the absolute-value evaluation of every entry.
    """
    q = np.asarray(q, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    if absolute:
        q, n = np.abs(q), np.abs(n)
    rho, mom, E = q[:, 0], q[:, 1:4], q[:, 4]
    g1 = GAMMA - 1.0
    mm = np.einsum("ij,ij->i", mom, mom)
    s = np.einsum("ij,ij->i", mom, n) / rho
    sg = 1.0 if absolute else -1.0  # sign of the terms that cancel
    p = g1 * (E + sg * 0.5 * mm / rho)
    ds_drho = sg * s / rho
    ds_dm = n / rho[:, None]
    dp_drho = g1 * 0.5 * mm / rho**2
    dp_dm = sg * g1 * mom / rho[:, None]
    dp_dE = g1
    M = len(q)
    J = np.zeros((M, 5, 5))
    J[:, 0, 1:4] = n
    for i in range(3):
        J[:, 1 + i, 0] = mom[:, i] * ds_drho + n[:, i] * dp_drho
        for j in range(3):
            J[:, 1 + i, 1 + j] = (s if i == j else 0.0) + mom[:, i] * ds_dm[:, j] + n[:, i] * dp_dm[:, j]
        J[:, 1 + i, 4] = n[:, i] * dp_dE
    J[:, 4, 0] = dp_drho * s + (E + p) * ds_drho
    J[:, 4, 1:4] = dp_dm * s[:, None] + (E + p)[:, None] * ds_dm
    J[:, 4, 4] = (1.0 + dp_dE) * s
    return J


def backward(n_vertices: int, edges: np.ndarray, geom: np.ndarray, q: np.ndarray, g_r: np.ndarray) -> np.ndarray:
    """g_q = (dr/dq)^T g_r, assembled from per-edge 5x5 Jacobians.

    dF/dq_u = J(q_u)/2 + sigma I/2, dF/dq_v = J(q_v)/2 - sigma I/2 and
    delta_e = a_e (g_r[u_e] - g_r[v_e]) is the upstream gradient of F_e.
    """
    edges = np.asarray(edges, dtype=np.int64)
    q = np.asarray(q, dtype=np.float64)
    g_r = np.asarray(g_r, dtype=np.float64)
    nrm, area = split_geom(geom)
    u, v = edges[:, 0], edges[:, 1]
    delta = area[:, None] * (g_r[u] - g_r[v])
    I = np.eye(5)[None]
    Ju = 0.5 * euler_jacobian(q[u], nrm) + 0.5 * SIGMA * I
    Jv = 0.5 * euler_jacobian(q[v], nrm) - 0.5 * SIGMA * I
    g_q = np.zeros((n_vertices, 5))
    np.add.at(g_q, u, np.einsum("ekj,ek->ej", Ju, delta))
    np.add.at(g_q, v, np.einsum("ekj,ek->ej", Jv, delta))
    return g_q


def backward_abs(n_vertices: int, edges: np.ndarray, geom: np.ndarray, q: np.ndarray, g_r: np.ndarray) -> np.ndarray:
    """Absolute-value evaluation of ``backward`` (tolerance floor)."""
    edges = np.asarray(edges, dtype=np.int64)
    g_r = np.abs(np.asarray(g_r, dtype=np.float64))
    nrm, area = split_geom(geom)
    u, v = edges[:, 0], edges[:, 1]
    delta = np.abs(area)[:, None] * (g_r[u] + g_r[v])
    I = np.eye(5)[None]
    Ju = 0.5 * euler_jacobian(q[u], nrm, absolute=True) + 0.5 * SIGMA * I
    Jv = 0.5 * euler_jacobian(q[v], nrm, absolute=True) + 0.5 * SIGMA * I
    g = np.zeros((n_vertices, 5))
    np.add.at(g, u, np.einsum("ekj,ek->ej", Ju, delta))
    np.add.at(g, v, np.einsum("ekj,ek->ej", Jv, delta))
    return g


def loss(n_vertices, edges, geom, q) -> float:
    """L = sum over vertices and components of r^2."""
    r = forward(n_vertices, edges, geom, q)
    return float((r * r).sum())
