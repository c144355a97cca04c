"""Pins for the Problem 2 input generator (bilinear elements for rotated
anisotropic diffusion): the assembled interior stencil equals the closed-form
Q1 stencil of a constant tensor K = [[a, b], [b, c]] on square elements,

    centre 4(a+c)/3;  E, W  -2a/3 + c/3;  N, S  a/3 - 2c/3;
    NE, SW  -(a+c)/6 - b/2;  NW, SE  -(a+c)/6 + b/2,

derived by hand from the bilinear basis (independent of the generator's
quadrature); K = I gives the standard 8/3, -1/3 stencil."""

import numpy as np
import pytest

from synth import anisotropic_problem, anisotropic_tensor, config, q1_stiffness


def _stencil(A, nx, ix, iy):
    row = A.getrow((ix - 1) + nx * (iy - 1)).toarray().ravel()
    out = {}
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            out[(dx, dy)] = row[(ix - 1 + dx) + nx * (iy - 1 + dy)]
    return out


@pytest.mark.parametrize("theta,eps", [(0.0, 1.0), (0.7, 1.0), (3 * np.pi / 16, 1e-3), (-0.4, 0.2)])
def test_interior_stencil_closed_form(theta, eps):
    nx = 9
    K = anisotropic_tensor(theta, eps)
    a, b, c = K[0, 0], K[0, 1], K[1, 1]
    A = q1_stiffness((nx, nx), K)
    st = _stencil(A, nx, 5, 5)
    want = {(0, 0): 4 * (a + c) / 3, (1, 0): -2 * a / 3 + c / 3, (-1, 0): -2 * a / 3 + c / 3,
            (0, 1): a / 3 - 2 * c / 3, (0, -1): a / 3 - 2 * c / 3,
            (1, 1): -(a + c) / 6 - b / 2, (-1, -1): -(a + c) / 6 - b / 2,
            (-1, 1): -(a + c) / 6 + b / 2, (1, -1): -(a + c) / 6 + b / 2}
    for k, v in want.items():
        assert st[k] == pytest.approx(v, rel=1e-12, abs=1e-14), k
    if eps == 1.0:
        assert st[(0, 0)] == pytest.approx(8 / 3) and st[(1, 1)] == pytest.approx(-1 / 3)


def test_tensor_and_matrix_properties():
    th = 3 * np.pi / 16
    K = anisotropic_tensor(th, 1e-3)
    np.testing.assert_allclose(np.linalg.eigvalsh(K), [1e-3, 1.0], rtol=1e-12)
    # the strong direction is (cos th, sin th): K v = v
    v = np.array([np.cos(th), np.sin(th)])
    np.testing.assert_allclose(K @ v, v, atol=1e-15)
    p = anisotropic_problem((12, 12), (2, 2))
    A = p.A
    assert (A != A.T).nnz == 0
    assert np.linalg.eigvalsh(A.toarray()).min() > 0
    # zero row sums away from the boundary, 9 entries per interior row
    rs = np.asarray(A.sum(axis=1)).ravel().reshape(12, 12)
    assert np.abs(rs[1:-1, 1:-1]).max() < 1e-12
    assert np.diff(A.indptr).max() == 9
    # positive off-diagonals are present (rotated anisotropy)
    assert (A.data > 0).sum() > A.shape[0]


def test_config_p2_shape():
    p = config("p2", scale=32)
    assert p.n == 32 * 32 and p.nparts == 16 and p.eta == 1 and p.n_fac == 2
    assert p.extra["eps"] == 1e-3
