"""Shape checks of the synthetic inputs (sizes, degree profiles, orientation)."""

import numpy as np

import gen
from gen.rmat import spmv_graph


def test_grid64_sizes():
    G = gen.grid2d(64, 64, seed=0)
    assert G["n"] == 4096 and len(G["edges"]) == 12_033
    E = G["edges"]
    assert (E[:, 0] < E[:, 1]).all()
    np.testing.assert_allclose(np.linalg.norm(G["geom"], axis=1), 1.0, rtol=1e-15)
    assert (np.diff(E[:, 0]) >= 0).all()  # default (u, v) order
    # seeded: same seed same ids, other seed other ids
    assert (gen.grid2d(64, 64, seed=0)["edges"] == E).all()
    assert not (gen.grid2d(64, 64, seed=1)["edges"] == E).all()


def test_tet32_sizes_and_degrees():
    T = gen.tet_mesh(32, 32, 32, seed=0)
    assert T["n"] == 196_608 and len(T["edges"]) == 387_072
    deg = np.bincount(T["edges"].ravel(), minlength=T["n"])
    vals, cnt = np.unique(deg, return_counts=True)
    assert dict(zip(vals.tolist(), cnt.tolist())) == {2: 192, 3: 11_904, 4: 184_512}


def test_tet_normals_point_from_u_to_v():
    T = gen.tet_mesh(5, 4, 3, seed=2)
    E, g, c = T["edges"], T["geom"], T["centroid"]
    assert (E[:, 0] < E[:, 1]).all()
    np.testing.assert_allclose(np.linalg.norm(g[:, :3], axis=1), 1.0, rtol=1e-12)
    assert (np.einsum("ij,ij->i", g[:, :3], c[E[:, 1]] - c[E[:, 0]]) > 0).all()
    assert (g[:, 3] > 0).all()
    m = 12 * 5 * 4 * 3 - 2 * (5 * 4 + 4 * 3 + 3 * 5)
    assert len(E) == m


def test_bfs_subgraph():
    S = gen.bfs_subgraph(gen.tet_mesh(6, 6, 6, seed=1), 1000)
    assert S["n"] == 1000
    assert S["edges"].max() < 1000 and (S["edges"][:, 0] < S["edges"][:, 1]).all()


def test_rmat_quadrant_frequencies():
    R = gen.rmat(scale=12, n_edges=200_000, seed=4)
    rows, cols = R["rows"].astype(np.int64), R["cols"].astype(np.int64)
    assert rows.max() < 4096 and cols.max() < 4096
    top_row = (rows >> 11) & 1
    top_col = (cols >> 11) & 1
    np.testing.assert_allclose(top_row.mean(), 0.19 + 0.05, atol=0.005)
    np.testing.assert_allclose(top_col.mean(), 0.19 + 0.05, atol=0.005)
    np.testing.assert_allclose((top_row & top_col).mean(), 0.05, atol=0.003)
    g = spmv_graph(R, R["shuffle"])
    assert g["edges"][:, 0].max() < 4096 and g["edges"][:, 1].min() >= 4096


def test_batch_sizes():
    B = gen.batch_graphs(16, seed=0)
    for i, g in enumerate(B):
        assert g["geom"].shape[1] == 4
        assert 0.4 * g["target_n"] <= g["n"] <= 2.5 * g["target_n"]
        assert g["dim"] == (2 if i % 2 == 0 else 3)
