"""The GPU eigensolver of the SVD clutter filter (Section 2.4.2: eigendecomposition of the
Casorati Gram S^H S) on Hermitian matrices whose spectra are known in closed form, so the
check does not go through the oracle:

  * a diagonal matrix in shuffled order: every Householder step meets a column that is
    already reduced (no reflection), and the eigenvalues are the diagonal itself;
  * 2x2 Hermitian blocks [[a, b], [conj(b), c]] coupling frames i and i + n/2: eigenvalues
    (a + c)/2 +- sqrt(((a - c)/2)^2 + |b|^2), eigenvectors inside each pair's plane;
  * a dense matrix H diag(lambda) H with H = I - 2 w w^H / (w^H w), a unitary reflection:
    the same eigenvalues, eigenvectors the columns of H.

Each at 200 frames (the reduction held in one workgroup's registers) and 400 (the
reduction through global memory)."""
import numpy as np
import pytest

from helpers import dev

pytestmark = pytest.mark.gpu

SIZES = [200, 400]


def _eig(gpu, A):
    import torch
    n = A.shape[0]
    ws = torch.empty(gpu.svd_workspace_size(1, n), dtype=torch.uint8, device='cuda')
    lam = torch.empty(n, dtype=torch.float64, device='cuda')
    vecs = torch.empty((n, n), dtype=torch.complex128, device='cuda')
    st = torch.full((1,), -1, dtype=torch.int32, device='cuda')
    gpu.hermitian_eig(dev(A), ws, lam, vecs, st)
    assert int(st.item()) == 0
    return lam.cpu().numpy(), vecs.cpu().numpy()


def _check_basis(A, lam, V, tol):
    n = A.shape[0]
    np.testing.assert_allclose(V.conj().T @ V, np.eye(n), atol=1e-10)
    np.testing.assert_allclose((V * lam) @ V.conj().T, A, atol=tol * np.abs(A).max())


@pytest.mark.parametrize('n', SIZES)
def test_eig_diagonal_shuffled(gpu, n):
    print('eig diagonal n', n, flush=True)
    rng = np.random.default_rng(900 + n)
    d = 10.0 ** np.linspace(6.0, -3.0, n)
    perm = rng.permutation(n)
    A = np.diag(d[perm]).astype(np.complex128)
    lam, V = _eig(gpu, A)
    np.testing.assert_allclose(lam, d, rtol=1e-9, atol=1e-12 * d[0])
    # eigenvector m is the unit vector of the frame that holds d[m]
    where = np.argsort(perm)   # where[m] = frame holding d[m]
    for K in (1, 5, 20):
        P = np.zeros((n, n))
        P[where[:K], where[:K]] = 1.0
        VK = V[:, :K]
        assert np.abs(VK @ VK.conj().T - P).max() < 1e-10
    _check_basis(A, lam, V, 1e-12)


@pytest.mark.parametrize('n', SIZES)
def test_eig_interleaved_2x2_blocks(gpu, n):
    print('eig 2x2 blocks n', n, flush=True)
    rng = np.random.default_rng(1900 + n)
    h = n // 2
    # block i = R diag(l1, l2) R^H, R a complex plane rotation; the 2h eigenvalues are a shuffled
    # geometric sequence (neighbours >= 3.5% apart, so no two pairs' vectors can mix)
    ev = 10.0 ** np.linspace(4.0, -2.0, n)
    lp = rng.permutation(ev).reshape(h, 2)
    th, ph = rng.uniform(0.1, 1.4, h), rng.uniform(0, 2 * np.pi, h)
    cs, sn = np.cos(th), np.sin(th)
    a = lp[:, 0] * cs ** 2 + lp[:, 1] * sn ** 2
    c = lp[:, 0] * sn ** 2 + lp[:, 1] * cs ** 2
    b = (lp[:, 0] - lp[:, 1]) * cs * sn * np.exp(1j * ph)
    # the quadratic formula gives the same pair (its smaller root by cancellation: to within
    # rounding of the larger)
    mid, rad = 0.5 * (a + c), np.sqrt((0.5 * (a - c)) ** 2 + np.abs(b) ** 2)
    qf = np.sort(np.stack([mid + rad, mid - rad], 1), 1)
    assert np.all(np.abs(qf - np.sort(lp, 1)) <= 1e-13 * lp.max(axis=1, keepdims=True))
    A = np.zeros((n, n), dtype=np.complex128)
    i = np.arange(h)
    A[i, i] = a
    A[i + h, i + h] = c
    A[i, i + h] = b
    A[i + h, i] = np.conj(b)
    lam, V = _eig(gpu, A)
    np.testing.assert_allclose(lam, ev, rtol=1e-9, atol=1e-12 * ev[0])
    # every eigenvector lies in the plane of one pair (i, i + h)
    mag = np.abs(V) ** 2
    pair = mag[:h] + mag[h:]
    assert np.all(pair.max(axis=0) > 1.0 - 1e-10)
    _check_basis(A, lam, V, 1e-11)


@pytest.mark.parametrize('n', SIZES)
def test_eig_reflected_diagonal(gpu, n):
    print('eig reflected diagonal n', n, flush=True)
    rng = np.random.default_rng(2900 + n)
    d = 10.0 ** np.linspace(4.0, -2.0, n)
    w = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    H = np.eye(n) - 2.0 * np.outer(w, w.conj()) / np.vdot(w, w).real
    A = (H * d) @ H.conj().T
    A = 0.5 * (A + A.conj().T)
    lam, V = _eig(gpu, A)
    np.testing.assert_allclose(lam, d, rtol=1e-9, atol=1e-12 * d[0])
    for K in (1, 5, 20):
        HK = H[:, :K]
        VK = V[:, :K]
        assert np.abs(VK @ VK.conj().T - HK @ HK.conj().T).max() < 1e-9
    _check_basis(A, lam, V, 1e-11)
