"""The singular-matrix error paths, forced from the host with well-formed
inputs (every kernel runs to its normal end; the singularity is detected in
the results and reported as QCD_ESINGULAR):

* an odd site whose clover block A(x) is singular: with c_sw = 1 the oracle
  gives A(x) = 1 + H(x) per site; H's two chirality blocks are Hermitian, so
  c_sw = -1 / lambda, lambda the most negative eigenvalue over the odd
  sites, makes one odd-site block 1 + c_sw H exactly singular (up to FP64
  rounding, far below the inverse's pivot threshold).  A slightly smaller
  c_sw is accepted;
* a deflation basis with one field zero on one block (loaded with
  deflation_set_phi): that block's diagonal little-operator block has a zero
  row and column, and its inverse (the block-Jacobi factor) fails.
"""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

DIMS, BLOCK = (8, 4, 4, 4), (2, 2, 2, 2)
KAPPA = 0.124


def _gpu():
    import torch
    import paper_1605_00564_amd as dfl
    return torch, dfl


def test_singular_odd_site_clover_block_is_reported():
    torch, dfl = _gpu()
    U = synth.gauge_field(DIMS, 0.4, 3)
    op = oracle.Operator(DIMS, U, KAPPA, 1.0, -1)
    V = op.V
    H = op.Am.reshape(V, 12, 12) - np.eye(12)[None]
    odd = np.array([sum(synth.coords(DIMS, i)) % 2 == 1 for i in range(V)])
    lam = min(np.linalg.eigvalsh(H[odd][:, :6, :6]).min(), np.linalg.eigvalsh(H[odd][:, 6:, 6:]).min())
    assert lam < 0
    csw = -1.0 / lam
    with pytest.raises(dfl.DflError) as e:
        dfl.Field(DIMS, BLOCK, KAPPA, csw, U)
    assert e.value.code == -5 and "clover" in str(e.value)
    dfl.Field(DIMS, BLOCK, KAPPA, 0.9 * csw, U).close()


def test_singular_little_operator_block_is_reported():
    torch, dfl = _gpu()
    U = synth.gauge_field(DIMS, 0.4, 3)
    fld = dfl.Field(DIMS, BLOCK, KAPPA, 1.0, U)
    d = dfl.Deflation(fld, Ns=4, ninv=1, seed=5, sap=dfl.SapParams(5, 4, 1))
    phi = d.get_phi()
    phi[3, 2] = 0            # field 2 vanishes on block 3
    with pytest.raises(dfl.DflError) as e:
        d.set_phi(phi)
    assert e.value.code == -5 and "little operator" in str(e.value)
    d.close()
    fld.close()
