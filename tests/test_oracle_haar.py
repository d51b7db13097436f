"""Pins of the oracle Haar operators (eq. intops, eq. intops_wav, eq. 1of4-4of4).

  * [I; J] is orthogonal: I I^T = J J^T = identity, I J^T = 0, I^T I + J^T J = identity;
  * the four 2D operators stacked are orthogonal, and one level reproduces the
    four pixel combinations (a+b+c+d)/2, (a-b+c-d)/2, (a+b-c-d)/2, (a-b-c+d)/2
    with a, b neighbours along x and a, c neighbours along y;
  * H_L (full packet tree) is orthogonal, the recursive transform equals the
    explicit matrix, and H_L^T undoes it;
  * a constant image c maps to 2^L c on the coarsest LL...L block and 0 elsewhere;
  * every row of H_L is a +-2^-L pattern on exactly one 2^L x 2^L pixel tile.
"""
import numpy as np
import pytest

from oracle import haar


@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_1d_scaling_and_wavelet_orthogonal(n):
    I, J = (a.toarray() for a in haar.intergrid_1d(n))
    e = np.eye(n // 2)
    assert np.allclose(I @ I.T, e, atol=1e-15)
    assert np.allclose(J @ J.T, e, atol=1e-15)
    assert np.allclose(I @ J.T, 0, atol=1e-15)
    assert np.allclose(I.T @ I + J.T @ J, np.eye(n), atol=1e-15)


@pytest.mark.parametrize("n", [2, 4, 8])
def test_2d_step_orthogonal_and_explicit(n):
    ops = haar.step_operators_2d(n)
    S = np.vstack([ops[k].toarray() for k in ("LL", "LH", "HL", "HH")])
    assert np.allclose(S @ S.T, np.eye(n * n), atol=1e-15)
    x = np.random.default_rng(0).standard_normal((n, n))
    c = haar.haar_step(x)
    h = n // 2
    a, b = x[0::2, 0::2], x[0::2, 1::2]      # b: x-neighbour of a
    cc, d = x[1::2, 0::2], x[1::2, 1::2]     # cc: y-neighbour of a
    assert np.allclose(c[:h, :h], (a + b + cc + d) / 2, atol=1e-15)
    assert np.allclose(c[:h, h:], (a - b + cc - d) / 2, atol=1e-15)
    assert np.allclose(c[h:, :h], (a + b - cc - d) / 2, atol=1e-15)
    assert np.allclose(c[h:, h:], (a - b - cc + d) / 2, atol=1e-15)


@pytest.mark.parametrize("n,L", [(4, 1), (8, 2), (8, 3), (16, 2), (16, 4)])
def test_packet_transform_orthogonal_and_consistent(n, L):
    H = haar.packet_matrix(n, L).toarray()
    assert np.allclose(H @ H.T, np.eye(n * n), atol=1e-14)
    x = np.random.default_rng(1).standard_normal((n, n))
    c = haar.packet_transform(x, L)
    assert np.allclose(c.ravel(), H @ x.ravel(), atol=1e-14)
    assert np.allclose(haar.packet_adjoint(c, L), x, atol=1e-14)
    y = np.random.default_rng(2).standard_normal((n, n))
    assert np.allclose(haar.packet_adjoint(y, L).ravel(), H.T @ y.ravel(), atol=1e-14)


@pytest.mark.parametrize("n,L", [(8, 1), (8, 3), (32, 2)])
def test_constant_image(n, L):
    c = haar.packet_transform(np.full((n, n), 3.0), L)
    cs = n >> L
    assert np.allclose(c[:cs, :cs], 3.0 * 2 ** L, atol=1e-13)
    c[:cs, :cs] = 0
    assert np.abs(c).max() < 1e-13


@pytest.mark.parametrize("n,L", [(8, 2), (16, 3)])
def test_rows_are_walsh_patterns_on_one_tile(n, L):
    H = haar.packet_matrix(n, L).toarray()
    T = 1 << L
    for q in range(n * n):
        row = H[q].reshape(n, n)
        nz = np.argwhere(np.abs(row) > 1e-14)
        assert len(nz) == T * T
        ty, tx = nz[0] // T
        assert (nz // T == (ty, tx)).all()
        assert np.allclose(np.abs(row[nz[:, 0], nz[:, 1]]), 2.0 ** -L, atol=1e-15)
        p, J = haar.subband_of(q // n, q % n, n, L)
        assert J == ty * (n >> L) + tx
