"""Pins of the dense primitives: Q-map algebra (eq. qij_epseps; remark after Def. def:deng;
proof of Thm thm:cemats; proof of Lemma thm:mu2), the harmonic mean identities of Lemma
thm:mu2 (eqs. sum_dagger_sum, harm_pinv), and the pseudo-inverse / generalized eigenvalue
primitives against LAPACK special cases."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.dense import genmax, harmonic, pinv_tau, q_half, q_transport, qmat, skew

rng = np.random.default_rng(11)


def _pts(m):
    return [rng.standard_normal(3) for _ in range(m)]


def _psd(n, rank=None):
    rank = n if rank is None else rank
    X = rng.standard_normal((n, rank))
    return X @ X.T


def test_skew_is_cross_product():
    t, r = rng.standard_normal(3), rng.standard_normal(3)
    assert np.allclose(skew(t) @ r, np.cross(t, r), atol=1e-15)


def test_q_maps_rigid_motion_between_points():
    # u(y) = d + y x r  <=>  (u(x_j), r) = Q^{i->j} (u(x_i), r)
    d, r = rng.standard_normal(3), rng.standard_normal(3)
    xi, xj = _pts(2)
    ui = np.concatenate([d + np.cross(xi, r), r])
    uj = np.concatenate([d + np.cross(xj, r), r])
    assert np.allclose(q_transport(xi, xj, 6) @ ui, uj, atol=1e-14)


def test_q_algebra_identities():
    xi, xj, xl, xI, xJ = _pts(5)
    k = 6
    # Q^ij Q^ij = Q^{i->j}  (Q^ij = sqrt(Q^{i->j}))
    assert np.allclose(q_half(xi, xj, k) @ q_half(xi, xj, k), q_transport(xi, xj, k), atol=1e-14)
    # composition Q^{i->j} Q^{j->l} = Q^{i->l}
    assert np.allclose(q_transport(xj, xl, k) @ q_transport(xi, xj, k), q_transport(xi, xl, k),
                       atol=1e-14)
    # Q^ji = (Q^ij)^{-1}
    assert np.allclose(q_half(xj, xi, k) @ q_half(xi, xj, k), np.eye(6), atol=1e-14)
    # Q^{IJ->ij} Q^IJ = Q^ij Q^{I->i}  with Q^{IJ->ij} = Q^ij Q^{I->i} Q^JI
    T = q_half(xi, xj, k) @ q_transport(xI, xi, k) @ q_half(xJ, xI, k)
    assert np.allclose(T @ q_half(xI, xJ, k), q_half(xi, xj, k) @ q_transport(xI, xi, k),
                       atol=1e-13)
    # Q^{i->l} Q^ji = Q^{j->l} Q^ij  (both map the midpoint of (i, j) to x_l)
    assert np.allclose(q_transport(xi, xl, k) @ q_half(xj, xi, k),
                       q_transport(xj, xl, k) @ q_half(xi, xj, k), atol=1e-13)
    # scalar case: Q = 1
    assert qmat(xi, 1).shape == (1, 1) and qmat(xi, 1)[0, 0] == 1.0


def test_midpoint_map_takes_coordinates_to_edge_midpoint():
    d, r = rng.standard_normal(3), rng.standard_normal(3)
    xi, xj = _pts(2)
    m = 0.5 * (xi + xj)
    ui = np.concatenate([d + np.cross(xi, r), r])
    assert np.allclose(q_half(xi, xj, 6) @ ui, np.concatenate([d + np.cross(m, r), r]),
                       atol=1e-14)


@pytest.mark.parametrize("ra,rb", [(6, 6), (3, 4), (2, 2), (1, 1), (0, 3), (5, 1)])
def test_harmonic_mean_identities(ra, rb):
    A, B = _psd(6, ra), _psd(6, rb)
    S = pinv_tau(A + B, 1e-12)
    H = harmonic(A, B, 1e-12)
    # eq. harm_pinv
    lhs = A @ S @ B @ S @ A + B @ S @ A @ S @ B
    scale = max(np.abs(A).max(), np.abs(B).max(), 1.0)
    assert np.allclose(lhs, A @ S @ B, atol=1e-9 * scale)
    # symmetric PSD, H(A, B) = H(B, A), H <= A and H <= B
    assert np.allclose(H, H.T, atol=1e-12 * scale)
    assert np.linalg.eigvalsh(H).min() > -1e-9 * scale
    assert np.allclose(H, harmonic(B, A, 1e-12), atol=1e-9 * scale)
    assert np.linalg.eigvalsh(A - H).min() > -1e-9 * scale
    # eq. sum_dagger_sum: ||x||_A = ||(A+B)^+(A+B) x||_A
    x = rng.standard_normal(6)
    y = S @ (A + B) @ x
    assert abs(x @ A @ x - y @ A @ y) < 1e-8 * scale * (x @ x)


def test_harmonic_scalar_closed_form():
    a, b = 3.0, 5.0
    assert abs(harmonic(np.array([[a]]), np.array([[b]]))[0, 0] - a * b / (a + b)) < 1e-15


def test_pinv_matches_lapack_and_drops_tau_kernel():
    X = _psd(6)
    assert np.allclose(pinv_tau(X), np.linalg.inv(X), rtol=1e-10, atol=1e-12)
    Y = _psd(6, 4)
    assert np.allclose(pinv_tau(Y), np.linalg.pinv(Y, rcond=1e-10, hermitian=True), atol=1e-10)
    # eigenvalue below tau * lambda_max is treated as zero
    U = np.linalg.qr(rng.standard_normal((6, 6)))[0]
    Z = U @ np.diag([1.0, 0.5, 0.2, 1e-3, 1e-12, 0.0]) @ U.T
    P = pinv_tau(Z, 1e-10)
    expect = U[:, :4] @ np.diag([1.0, 2.0, 5.0, 1e3]) @ U[:, :4].T
    assert np.allclose(P, expect, atol=1e-8)
    assert np.all(pinv_tau(np.zeros((3, 3))) == 0)


def test_genmax_spd_matches_lapack_generalized_eigensolver():
    L, R = _psd(6), _psd(6)
    assert abs(genmax(L, R) - sla.eigh(L, R, eigvals_only=True).max()) < 1e-9 * genmax(L, R)


def test_genmax_singular_pencils():
    U = np.linalg.qr(rng.standard_normal((6, 6)))[0]
    R = U[:, :4] @ np.diag([4.0, 3.0, 2.0, 1.0]) @ U[:, :4].T
    L_in = U[:, :2] @ np.diag([8.0, 1.0]) @ U[:, :2].T     # range(L) inside range(R)
    assert abs(genmax(L_in, R) - 2.0) < 1e-12
    L_out = L_in + 1e-3 * np.outer(U[:, 5], U[:, 5])       # positive on null(R)
    assert genmax(L_out, R) == float("inf")
    assert genmax(np.zeros((6, 6)), R) == 0.0
    # smallest mu with L <= mu R: check the bound is tight
    mu = genmax(L_in, R)
    assert np.linalg.eigvalsh(mu * R - L_in).min() > -1e-12
    assert np.linalg.eigvalsh(0.99 * mu * R - L_in).min() < 0
