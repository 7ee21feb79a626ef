"""Oracle for source and sink smearing (section 2.3: Gaussian smearing with
APE-smeared gauge links in the Laplacian, at source and sink).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy, FP64.
The paper takes its smearing parameters from earlier work, so they are
inputs here.  Readings (the paper gives no formulas):

* APE smearing of the spatial links, n_iter times:
      U'_i(x) = P[ (1 - alpha) U_i(x) + (alpha / 4) sum_{j != i, spatial} (
                   U_j(x) U_i(x + j) U_j(x + i)^+
                 + U_j(x - j)^+ U_i(x - j) U_j(x - j + i) ) ],
  with P the projection onto SU(3): the unitary polar factor W of V
  (from its singular value decomposition V = A S B^+, W = A B^+), divided
  by a cube root of its determinant, det(W)^(1/3) = exp(i arg(det W) / 3)
  with arg in (-pi, pi].  Time links are not smeared.
* Gaussian smearing with the smeared spatial links, n_iter times:
      psi'(x) = [ psi(x) + kappa_G sum_{i spatial} ( U'_i(x) psi(x + i)
                 + U'_i(x - i)^+ psi(x - i) ) ] / (1 + 6 kappa_G),
  acting on colour only (every spin component alike) and within each
  timeslice; spatial boundaries are periodic.
"""

from __future__ import annotations

import numpy as np


def _shift(dims, f, mu, step):
    """f(x + step mu) for a site field f[V, ...]."""
    sh = f.reshape(tuple(dims) + f.shape[1:])
    return np.roll(sh, -step, axis=mu).reshape(f.shape)


def project_su3(V):
    """Polar factor of each 3x3 matrix divided by a cube root of its determinant."""
    A, _, Bh = np.linalg.svd(V)
    W = A @ Bh
    ph = np.angle(np.linalg.det(W))
    return W * np.exp(-1j * ph / 3)[..., None, None]


def ape_smear(dims, U, alpha, n_iter):
    """Spatially APE-smeared links; U[V, 4, 3, 3] -> same shape (time links copied)."""
    U = np.array(U, dtype=np.complex128, copy=True)
    dag = lambda m: np.conj(np.swapaxes(m, -1, -2))
    for _ in range(n_iter):
        new = U.copy()
        for i in (1, 2, 3):
            S = np.zeros_like(U[:, i])
            for j in (1, 2, 3):
                if j == i:
                    continue
                Uj, Ui = U[:, j], U[:, i]
                up = Uj @ _shift(dims, Ui, j, 1) @ dag(_shift(dims, Uj, i, 1))
                Ujm = _shift(dims, Uj, j, -1)
                dn = dag(Ujm) @ _shift(dims, Ui, j, -1) @ _shift(dims, _shift(dims, Uj, j, -1), i, 1)
                S += up + dn
            new[:, i] = project_su3((1 - alpha) * U[:, i] + 0.25 * alpha * S)
        U = new
    return U


def gauss_smear(dims, U, psi, kappa, n_iter):
    """Gaussian smearing of psi[V, 4, 3] (or [n, V, 4, 3]) with links U[V, 4, 3, 3]."""
    psi = np.asarray(psi, dtype=np.complex128)
    if psi.ndim == 4:
        return np.stack([gauss_smear(dims, U, p, kappa, n_iter) for p in psi])
    dag = lambda m: np.conj(np.swapaxes(m, -1, -2))
    for _ in range(n_iter):
        acc = psi.copy()
        for i in (1, 2, 3):
            fwd = np.einsum("xab,xsb->xsa", U[:, i], _shift(dims, psi, i, 1))
            bwd = np.einsum("xab,xsb->xsa", _shift(dims, dag(U[:, i]), i, -1), _shift(dims, psi, i, -1))
            acc += kappa * (fwd + bwd)
        psi = acc / (1 + 6 * kappa)
    return psi
