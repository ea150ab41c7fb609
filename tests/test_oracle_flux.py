"""Pins for the oracle's FLUX5 forward and adjoint and for SpMV.

The interaction formula is this project's reading (the paper prints none), so
it is pinned by properties mathematics fixes for any consistent Euler normal
flux with central dissipation: antisymmetry, conservation, free-stream
preservation on closed cells, rotation invariance, degree-1 homogeneity
(f = J q), the textbook eigenvalues of the flux Jacobian, finite differences
and the dot-product test.  SpMV is pinned by scipy.sparse.
"""

import numpy as np
import pytest
import scipy.sparse as sp

import gen
from oracle import flux, spmv

RNG = np.random.default_rng(1234)


def _states(M, rng=RNG, lo=0.5, hi=1.5):
    return rng.uniform(lo, hi, size=(M, 5))


def _unit(M, rng=RNG, dim=3):
    v = rng.standard_normal((M, 3))
    if dim == 2:
        v[:, 2] = 0
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_antisymmetry():
    qu, qv, n = _states(100), _states(100), _unit(100)
    np.testing.assert_allclose(flux.edge_flux(qv, qu, -n), -flux.edge_flux(qu, qv, n), rtol=1e-14, atol=1e-14)


def test_pressure_equilibrium_closed_form():
    """Zero momentum and equal pressure: mass and energy move by dissipation
    only, momentum by pressure alone: F = (sigma (rho_u - rho_v)/2, p n, 0)."""
    M = 50
    qu, qv, n = _states(M), _states(M), _unit(M)
    qu[:, 1:4] = 0
    qv[:, 1:4] = 0
    qv[:, 4] = qu[:, 4]
    F = flux.edge_flux(qu, qv, n)
    p = (flux.GAMMA - 1) * qu[:, 4]
    np.testing.assert_allclose(F[:, 0], 0.5 * flux.SIGMA * (qu[:, 0] - qv[:, 0]), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(F[:, 1:4], p[:, None] * n, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(F[:, 4], 0, atol=1e-15)


def test_rotation_invariance():
    """Rotating momentum and normal together rotates the momentum flux."""
    M = 40
    q, n = _states(M), _unit(M)
    A = np.linalg.qr(RNG.standard_normal((3, 3)))[0]
    qr = q.copy()
    qr[:, 1:4] = q[:, 1:4] @ A.T
    f = flux.euler_flux(q, n)
    fr = flux.euler_flux(qr, n @ A.T)
    np.testing.assert_allclose(fr[:, [0, 4]], f[:, [0, 4]], rtol=1e-13)
    np.testing.assert_allclose(fr[:, 1:4], f[:, 1:4] @ A.T, rtol=1e-12, atol=1e-13)


def test_homogeneity_and_jacobian_identity():
    """The Euler flux is homogeneous of degree one, so f(q) = J(q) q."""
    M = 60
    q, n = _states(M), _unit(M)
    np.testing.assert_allclose(flux.euler_flux(3.7 * q, n), 3.7 * flux.euler_flux(q, n), rtol=1e-12, atol=1e-13)
    J = flux.euler_jacobian(q, n)
    np.testing.assert_allclose(np.einsum("ekj,ej->ek", J, q), flux.euler_flux(q, n), rtol=1e-12, atol=1e-13)


def test_jacobian_eigenvalues_textbook():
    """Eigenvalues of the normal flux Jacobian: u_n - c, u_n (x3), u_n + c, c^2 = gamma p / rho."""
    M = 30
    q, n = _states(M), _unit(M)
    q[:, 1:4] *= 0.2  # keep the pressure positive
    J = flux.euler_jacobian(q, n)
    rho, mom, E = q[:, 0], q[:, 1:4], q[:, 4]
    p = (flux.GAMMA - 1) * (E - 0.5 * (mom * mom).sum(1) / rho)
    assert (p > 0).all()
    un = (mom * n).sum(1) / rho
    c = np.sqrt(flux.GAMMA * p / rho)
    for e in range(M):
        ev = np.sort(np.linalg.eigvals(J[e]).real)
        np.testing.assert_allclose(ev, np.sort([un[e] - c[e], un[e], un[e], un[e], un[e] + c[e]]), atol=1e-9)


def test_jacobian_finite_differences():
    M = 20
    q, n = _states(M), _unit(M)
    J = flux.euler_jacobian(q, n)
    h = 1e-6
    for j in range(5):
        dq = np.zeros_like(q)
        dq[:, j] = h
        fd = (flux.euler_flux(q + dq, n) - flux.euler_flux(q - dq, n)) / (2 * h)
        np.testing.assert_allclose(J[:, :, j], fd, rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("dim", [2, 3])
def test_conservation_and_free_stream(dim):
    if dim == 2:
        G = gen.grid2d(12, 9, seed=3)
    else:
        G = gen.tet_mesh(4, 3, 5, seed=3)
    n, E, geom = G["n"], G["edges"], G["geom"]
    q = _states(n)
    r = flux.forward(n, E, geom, q)
    nrm, area = flux.split_geom(geom)
    scale = np.abs(flux.edge_flux(q[E[:, 0]], q[E[:, 1]], nrm) * area[:, None]).sum()
    assert np.abs(r.sum(0)).max() <= 1e-12 * scale  # conservation
    # uniform state: interior vertices (full degree) see zero net flux, boundary ones do not
    qb = np.tile(_states(1), (n, 1))
    rb = flux.forward(n, E, geom, qb)
    deg = np.bincount(E.ravel(), minlength=n)
    full = 6 if dim == 2 else 4
    assert np.abs(rb[deg == full]).max() <= 1e-13
    assert np.abs(rb[deg < full]).max(axis=1).min() > 1e-6


def test_forward_abs_floor_and_dt():
    G = gen.tet_mesh(3, 3, 3, seed=1)
    n, E, geom = G["n"], G["edges"], G["geom"]
    q = _states(n)
    r, qn = flux.forward(n, E, geom, q, dt=0.01)
    A = flux.forward_abs(n, E, geom, q)
    assert (A >= np.abs(r) - 1e-15).all()
    np.testing.assert_allclose(qn, q + 0.01 * r, rtol=0, atol=0)


def _subgraph_1k():
    return gen.bfs_subgraph(gen.tet_mesh(8, 8, 8, seed=5), 1000)


# One 2D edge (area 1) worked out by hand: n = (0.6, -0.8), q_u = (1, -1, 2, 0, 3),
# q_v = (2, 2, -2, 0, 5), gamma = 1.4, sigma = 1.
#   signed: s_u = (-0.6 - 1.6)/1 = -2.2, p_u = 0.4 (3 - 5/2) = 0.2,
#           f_u = (-2.2, 2.2 + 0.12, -4.4 - 0.16, 0, 3.2 * -2.2) = (-2.2, 2.32, -4.56, 0, -7.04);
#           s_v = (1.2 + 1.6)/2 = 1.4, p_v = 0.4 (5 - 8/4) = 1.2,
#           f_v = (2.8, 2.8 + 0.72, -2.8 - 0.96, 0, 6.2 * 1.4) = (2.8, 3.52, -3.76, 0, 8.68);
#           F = (f_u + f_v)/2 - (q_v - q_u)/2 = (0.3, 2.92, -4.16, 0, 0.82) - (0.5, 1.5, -2, 0, 1)
#             = (-0.2, 1.42, -2.16, 0, -0.18); r_u = F, r_v = -F.
#   absolute-value evaluation (|q|, |n| = (0.6, 0.8), every minus a plus):
#           |q_u| = (1, 1, 2, 0, 3): s = 0.6 + 1.6 = 2.2, p = 0.4 (3 + 5/2) = 2.2,
#             f = (2.2, 2.2 + 1.32, 4.4 + 1.76, 0, 5.2 * 2.2) = (2.2, 3.52, 6.16, 0, 11.44);
#           |q_v| = (2, 2, 2, 0, 5): s = (1.2 + 1.6)/2 = 1.4, p = 0.4 (5 + 8/4) = 2.8,
#             f = (2.8, 2.8 + 1.68, 2.8 + 2.24, 0, 7.8 * 1.4) = (2.8, 4.48, 5.04, 0, 10.92);
#           A = (f_u + f_v)/2 + (|q_v| + |q_u|)/2 = (2.5, 4, 5.6, 0, 11.18) + (1.5, 1.5, 2, 0, 4)
#             = (4, 5.5, 7.6, 0, 15.18) at both endpoints.
#   adjoint floor with g_r[u] = (1, -1, 1, -1, 1), g_r[v] = 0, so |delta| = (1, 1, 1, 1, 1):
#           B_w = (J_abs(q_w)/2 + I/2)^T |delta| = (column sums of J_abs(q_w) + 1) / 2, with
#           J_abs(|q_u|) rows (0, .6, .8, 0, 0), (2.8, 3.04, 1.28, 0, .24), (5.2, 1.52, 4.44, 0, .32),
#             (0, 0, 0, 2.2, 0), (13.64, 4, 5.92, 0, 3.08): column sums (21.64, 9.16, 12.44, 2.2, 3.64);
#           J_abs(|q_v|) rows (0, .6, .8, 0, 0), (1.64, 2.24, 1.04, 0, .24), (1.72, .92, 2.52, 0, .32),
#             (0, 0, 0, 1.4, 0), (6.02, 2.9, 3.68, 0, 1.96): column sums (9.38, 6.66, 8.04, 1.4, 2.52).
_E1 = np.array([[0, 1]])
_G1 = np.array([[0.6, -0.8]])
_Q1 = np.array([[1.0, -1.0, 2.0, 0.0, 3.0], [2.0, 2.0, -2.0, 0.0, 5.0]])


def test_single_edge_forward_hand_derived():
    F = np.array([-0.2, 1.42, -2.16, 0.0, -0.18])
    r = flux.forward(2, _E1, _G1, _Q1)
    assert np.allclose(r, np.stack([F, -F]), rtol=0, atol=1e-14)


# The same edge in 3D, turned so that the normal has a z component and scaled by an area:
# n = (0, 0.6, -0.8), a = 2, q_u = (1, 0, -1, 2, 3), q_v = (2, 0, 2, -2, 5).  The momenta
# move with the normal (m2, m3 take the roles of m1, m2 above), so m.n and |m|^2 are as
# before: s_u = -2.2, p_u = 0.2, s_v = 1.4, p_v = 1.2,
#   f_u = (-2.2, 0, 2.2 + 0.12, -4.4 - 0.16, -7.04) = (-2.2, 0, 2.32, -4.56, -7.04),
#   f_v = (2.8, 0, 2.8 + 0.72, -2.8 - 0.96, 8.68) = (2.8, 0, 3.52, -3.76, 8.68),
#   a [(f_u + f_v)/2 - (q_v - q_u)/2] = 2 [(0.3, 0, 2.92, -4.16, 0.82) - (0.5, 0, 1.5, -2, 1)]
#     = (-0.4, 0, 2.84, -4.32, -0.36).
# The area multiplies the dissipation as well as the Euler flux: leaving it off the
# dissipation would give (0.1, 0, 4.34, -6.32, 0.64).


def test_single_edge_3d_with_area_hand_derived():
    q = np.array([[1.0, 0.0, -1.0, 2.0, 3.0], [2.0, 0.0, 2.0, -2.0, 5.0]])
    geom = np.array([[0.0, 0.6, -0.8, 2.0]])
    F = np.array([-0.4, 0.0, 2.84, -4.32, -0.36])
    assert np.allclose(flux.forward(2, _E1, geom, q), np.stack([F, -F]), rtol=0, atol=1e-14)


def test_single_edge_abs_floors_hand_derived():
    """Pins the tolerance floors themselves: a floor that drops a term, keeps a sign or is
    inflated by any factor misses these values (so an elementwise parity check cannot be
    loosened through its floor)."""
    A = np.array([4.0, 5.5, 7.6, 0.0, 15.18])
    assert np.allclose(flux.forward_abs(2, _E1, _G1, _Q1), np.stack([A, A]), rtol=0, atol=1e-13)
    g_r = np.array([[1.0, -1.0, 1.0, -1.0, 1.0], [0.0] * 5])
    Bu = (np.array([21.64, 9.16, 12.44, 2.2, 3.64]) + 1.0) / 2
    Bv = (np.array([9.38, 6.66, 8.04, 1.4, 2.52]) + 1.0) / 2
    assert np.allclose(flux.backward_abs(2, _E1, _G1, _Q1, g_r), np.stack([Bu, Bv]), rtol=0, atol=1e-13)


def test_adjoint_matches_finite_differences_on_1k_cells():
    """FP64 central differences of L = sum r^2 with h_i = 1e-6 max(1, |q_i|)."""
    G = _subgraph_1k()
    n, E, geom = G["n"], G["edges"], G["geom"]
    assert n == 1000
    q = _states(n, np.random.default_rng(9))
    r = flux.forward(n, E, geom, q)
    g = flux.backward(n, E, geom, q, 2.0 * r)
    rng = np.random.default_rng(10)
    idx = rng.choice(n * 5, size=400, replace=False)  # 400 of the 5000 components
    fd = np.empty(len(idx))
    for t, flat in enumerate(idx):
        i, c = divmod(int(flat), 5)
        h = 1e-6 * max(1.0, abs(q[i, c]))
        qp, qm = q.copy(), q.copy()
        qp[i, c] += h
        qm[i, c] -= h
        fd[t] = (flux.loss(n, E, geom, qp) - flux.loss(n, E, geom, qm)) / (2 * h)
    an = g.reshape(-1)[idx]
    assert np.linalg.norm(an - fd) <= 1e-6 * np.linalg.norm(fd)


def test_adjoint_dot_product():
    """<J dq, lam> = <dq, J^T lam> with J = dr/dq by directional differences."""
    G = gen.tet_mesh(3, 4, 3, seed=2)
    n, E, geom = G["n"], G["edges"], G["geom"]
    rng = np.random.default_rng(11)
    q = _states(n, rng)
    lam = rng.standard_normal((n, 5))
    dq = rng.standard_normal((n, 5))
    h = 1e-6
    Jdq = (flux.forward(n, E, geom, q + h * dq) - flux.forward(n, E, geom, q - h * dq)) / (2 * h)
    lhs = (Jdq * lam).sum()
    rhs = (dq * flux.backward(n, E, geom, q, lam)).sum()
    assert abs(lhs - rhs) <= 1e-7 * abs(rhs)


def test_adjoint_matches_torch_autograd():
    """Second check: FP64 autograd of a torch transcription of the forward."""
    torch = pytest.importorskip("torch")
    G = gen.grid2d(7, 6, seed=4)
    n, E, geom = G["n"], G["edges"], G["geom"]
    rng = np.random.default_rng(12)
    q = _states(n, rng)
    gr = rng.standard_normal((n, 5))
    nrm, area = flux.split_geom(geom)
    Q = torch.tensor(q, dtype=torch.float64, requires_grad=True)
    N = torch.tensor(nrm)
    Ar = torch.tensor(area)[:, None]
    u, v = torch.tensor(E[:, 0].astype(np.int64)), torch.tensor(E[:, 1].astype(np.int64))

    def f(qq):
        rho, mom, En = qq[:, 0], qq[:, 1:4], qq[:, 4]
        s = (mom * N).sum(1) / rho
        p = (flux.GAMMA - 1) * (En - 0.5 * (mom * mom).sum(1) / rho)
        return torch.cat([(rho * s)[:, None], mom * s[:, None] + p[:, None] * N, ((En + p) * s)[:, None]], 1)

    F = (0.5 * (f(Q[u]) + f(Q[v])) - 0.5 * flux.SIGMA * (Q[v] - Q[u])) * Ar
    r = torch.zeros(n, 5, dtype=torch.float64).index_add(0, u, F).index_add(0, v, -F)
    (r * torch.tensor(gr)).sum().backward()
    np.testing.assert_allclose(flux.backward(n, E, geom, q, gr), Q.grad.numpy(), rtol=1e-11, atol=1e-12)


def test_backward_abs_floor():
    G = gen.grid2d(5, 5, seed=1)
    n, E, geom = G["n"], G["edges"], G["geom"]
    q = _states(n)
    gr = RNG.standard_normal((n, 5))
    assert (flux.backward_abs(n, E, geom, q, gr) >= np.abs(flux.backward(n, E, geom, q, gr)) - 1e-14).all()


# ---------------------------------------------------------------- SpMV

def test_spmv_matches_scipy_with_duplicates():
    R = gen.rmat(scale=10, n_edges=20_000, seed=3)
    G = gen.rmat.__module__  # noqa: F841  (module import check)
    from gen.rmat import spmv_graph

    g = spmv_graph(R)
    y = spmv.forward(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"])
    A = sp.coo_matrix((R["w"].astype(np.float64), (R["rows"], R["cols"])), shape=(R["n_y"], R["n_x"]))
    np.testing.assert_allclose(y, A @ R["x"].astype(np.float64), rtol=1e-12, atol=1e-12)
    dup = len(R["rows"]) - len(np.unique(R["rows"].astype(np.int64) * R["n_x"] + R["cols"]))
    assert dup > 0  # duplicates present and summed
    i = int(R["rows"][0])
    yi, ai = spmv.row(R["n_x"], g["edges"], g["w"], R["x"], i)
    assert abs(yi - y[i]) <= 1e-12 * ai
    assert (spmv.forward_abs(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"]) >= np.abs(y) - 1e-12).all()


def test_spmv_adjoint_matches_scipy_transpose_and_dot_product():
    """g_x = A^T g_y against scipy's transpose product (duplicates summed); <A x, g> = <x, A^T g>;
    the weight gradient against central differences of <g_y, A(w) x> (linear in w, so exact up to
    rounding)."""
    from gen.rmat import spmv_graph

    R = gen.rmat(scale=9, n_edges=3000, seed=4)
    g = spmv_graph(R)
    n_x, n_y = R["n_x"], R["n_y"]
    j = g["edges"][:, 0]
    i = g["edges"][:, 1] - n_x
    w = g["w"].astype(np.float64)
    A = sp.coo_matrix((w, (i, j)), shape=(n_y, n_x)).tocsr()
    rng = np.random.default_rng(0)
    gy = rng.standard_normal(n_y)
    x = R["x"].astype(np.float64)
    g_x, g_w = spmv.backward(n_x, n_y, g["edges"], g["w"], x, gy)
    assert np.allclose(g_x, A.T @ gy, rtol=1e-12, atol=1e-12)
    y = spmv.forward(n_x, n_y, g["edges"], g["w"], x)
    assert abs(y @ gy - x @ g_x) <= 1e-10 * (np.abs(y) @ np.abs(gy) + 1)
    for e in rng.choice(len(w), 25, replace=False):
        h = 1e-3
        wp, wm = w.copy(), w.copy()
        wp[e] += h
        wm[e] -= h
        fd = (spmv.forward(n_x, n_y, g["edges"], wp, x) @ gy - spmv.forward(n_x, n_y, g["edges"], wm, x) @ gy) / (2 * h)
        assert abs(fd - g_w[e]) <= 1e-8 * (1 + abs(g_w[e]))
    ax, aw = spmv.backward_abs(n_x, n_y, g["edges"], g["w"], x, gy)
    assert (ax >= np.abs(g_x) - 1e-12).all() and (aw >= np.abs(g_w) - 1e-12).all()
