"""Pins of the oracle's quadrature-assembled graph (Sec. 2.2, eqs. for m_i,
m_ij, c_ij and the unit_normal_vector integrals) against closed forms of the
uniform Q1 element and the identities the paper states for them."""
import numpy as np
import pytest

from oracle import oracle as O


def _entry(g, i, j):
    for e in range(g.row_ptr[i], g.row_ptr[i + 1]):
        if g.col[e] == j:
            return e
    raise KeyError((i, j))


@pytest.fixture(scope="module")
def g2():
    # 7 x 6 nodes on [0, 1.2] x [0, 1.0]: h = 0.2 both ways
    return O.Graph(2, (7, 6), (0.0, 0.0), (1.2, 1.0), (False, False))


@pytest.fixture(scope="module")
def g3():
    # h = 0.25 in every direction; y periodic
    return O.Graph(3, (5, 4, 6), (0.0, 0.0, 0.0), (1.0, 1.0, 1.25),
                   (False, True, False))


def test_closed_form_2d_interior(g2):
    h = 0.2
    nx = 7
    i = 3 + nx * 2  # interior node
    assert np.isclose(g2.mi[i], h * h, rtol=1e-14)
    assert np.isclose(g2.mij[_entry(g2, i, i)], 4 * h * h / 9, rtol=1e-14)
    assert np.isclose(g2.mij[_entry(g2, i, i + 1)], h * h / 9, rtol=1e-14)
    assert np.isclose(g2.mij[_entry(g2, i, i + 1 + nx)], h * h / 36, rtol=1e-14)
    e = _entry(g2, i, i + 1)
    assert np.allclose(g2.cij[:, e], [h / 3, 0.0], atol=1e-16)
    e = _entry(g2, i, i - nx)
    assert np.allclose(g2.cij[:, e], [0.0, -h / 3], atol=1e-16)
    e = _entry(g2, i, i + 1 + nx)
    assert np.allclose(g2.cij[:, e], [h / 12, h / 12], atol=1e-16)
    e = _entry(g2, i, i - 1 + nx)
    assert np.allclose(g2.cij[:, e], [-h / 12, h / 12], atol=1e-16)
    assert np.allclose(g2.cij[:, _entry(g2, i, i)], 0.0, atol=1e-16)
    assert g2.row_ptr[i + 1] - g2.row_ptr[i] == 9


def test_closed_form_2d_wall_and_corner(g2):
    h = 0.2
    nx = 7
    i = 3  # bottom wall, interior in x
    assert np.isclose(g2.mi[i], h * h / 2, rtol=1e-14)
    assert np.allclose(g2.cij[:, _entry(g2, i, i)], [0.0, -h / 3], atol=1e-16)
    assert np.allclose(g2.bnd[:, i], [0.0, -h], atol=1e-16)
    assert g2.row_ptr[i + 1] - g2.row_ptr[i] == 6
    c = 0  # corner
    assert np.isclose(g2.mi[c], h * h / 4, rtol=1e-14)
    assert np.allclose(g2.bnd[:, c], [-h / 2, -h / 2], atol=1e-16)
    assert g2.row_ptr[c + 1] - g2.row_ptr[c] == 4
    assert g2.on_wall[i] == 1 and g2.on_wall[c] == 1 and g2.on_wall[3 + nx * 2] == 0


def test_closed_form_3d_interior(g3):
    h = 0.25
    nx, ny = 5, 4
    i = 2 + nx * (1 + ny * 2)
    assert np.isclose(g3.mi[i], h ** 3, rtol=1e-14)
    e = _entry(g3, i, i + 1)
    assert np.allclose(g3.cij[:, e], [2 * h * h / 9, 0, 0], atol=1e-16)
    e = _entry(g3, i, i + 1 + nx)
    assert np.allclose(g3.cij[:, e], [h * h / 18, h * h / 18, 0], atol=1e-16)
    e = _entry(g3, i, i + 1 + nx + nx * ny)
    assert np.allclose(g3.cij[:, e], [h * h / 72] * 3, atol=1e-16)
    assert g3.row_ptr[i + 1] - g3.row_ptr[i] == 27


@pytest.mark.parametrize("name", ["g2", "g3"])
def test_identities(name, request):
    g = request.getfixturevalue(name)
    N, dim = g.N, g.dim
    row = np.repeat(np.arange(N), np.diff(g.row_ptr))
    scale = np.abs(g.cij).max()
    # sum_j c_ij = 0 for every i (partition of unity)
    for k in range(dim):
        s = np.bincount(row, weights=g.cij[k], minlength=N)
        assert np.abs(s).max() < 1e-14 * scale
    # m_i = sum_j m_ij
    assert np.allclose(np.bincount(row, weights=g.mij, minlength=N), g.mi,
                       rtol=1e-14, atol=0)
    # c_ij + c_ji = int_dOmega phi_i phi_j n  (zero unless both on the wall)
    assert np.abs(g.cij + g.cij[:, g.tr] - g.bpair).max() < 1e-14 * scale
    both_wall = (g.on_wall[row] == 1) & (g.on_wall[g.col] == 1)
    assert np.abs(g.bpair[:, ~both_wall]).max() == 0.0
    # sum_i c_ij = int_dOmega phi_j n
    for k in range(dim):
        s = np.bincount(g.col, weights=g.cij[k], minlength=N)
        assert np.abs(s - g.bnd[k]).max() < 1e-14 * scale
    # sum_i m_i = |Omega|
    if dim == 2:
        assert np.isclose(g.mi.sum(), 1.2 * 1.0, rtol=1e-14)
    else:
        assert np.isclose(g.mi.sum(), 1.0 * 1.0 * 1.25, rtol=1e-14)
    # transpose map is an involution onto (j, i)
    assert np.array_equal(g.tr[g.tr], np.arange(g.nnz))
    assert np.array_equal(g.col[g.tr], row)
    # symmetry of the consistent mass matrix
    assert np.array_equal(g.mij, g.mij[g.tr])


def test_periodic_graph_is_antisymmetric():
    g = O.Graph(2, (6, 5), (0, 0), (1.0, 1.0), (True, True))
    assert np.abs(g.cij + g.cij[:, g.tr]).max() < 1e-16
    assert np.all(np.diff(g.row_ptr) == 9)
    assert np.isclose(g.mi.sum(), 1.0, rtol=1e-14)
    assert not g.on_wall.any()


def test_invalid_meshes():
    with pytest.raises(ValueError):
        O.Graph(2, (2, 5), (0, 0), (1, 1), (True, False))
    with pytest.raises(ValueError):
        O.Graph(2, (1, 5), (0, 0), (1, 1), (False, False))
