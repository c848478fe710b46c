"""SVQB's eigenvalue floor (Sec. 4.2's SVQB: M = U L U^T, Z = U L^{-1/2}
U^T; eigenvalues below the floor u lambda_max, 2^-104 lambda_max in DD,
are lifted to it so that a rank-deficient block still gives a finite Z):
borth_info.svqb_lifted reports the largest number of eigenvalues one pass
lifted.  Diagonal M has its eigenvalues on the diagonal exactly, so the
expected count is known; a block with an exactly zero column has an exactly
zero Gram row and column in every pass."""
import numpy as np
import pytest

import synth
from gpu_common import dev, lib, note, torch_gpu


@pytest.mark.gpu
@pytest.mark.parametrize("dd", [False, True])
def test_factor_reports_lifted_eigenvalues(dd):
    borth = lib()
    torch_gpu()
    below = 1e-40 if dd else 1e-20   # under 2^-104 (4.9e-32) / u (1.1e-16) times lambda_max = 1
    above = 1e-28 if dd else 1e-12
    lo = (lambda M: dev(np.zeros_like(M))) if dd else (lambda M: None)
    M = np.diag([1.0, below, 0.0, 0.5])
    Z, _, _, info = borth.factor(dev(M), lo(M), fact="svqb")
    note("svqb lift", dd, info)
    assert info.status == 0 and info.svqb_lifted == 2
    assert np.isfinite(Z.cpu().numpy()).all()
    M = np.diag([1.0, above, 0.25, 0.5])
    _, _, _, info = borth.factor(dev(M), lo(M), fact="svqb")
    assert info.status == 0 and info.svqb_lifted == 0
    _, _, _, info = borth.factor(dev(M), lo(M), fact="chol")
    assert info.status == 0 and info.svqb_lifted == 0


@pytest.mark.gpu
@pytest.mark.parametrize("gram", ["f64", "dd"])
def test_orthonormalize_reports_lifted_eigenvalues(gram):
    borth = lib()
    torch_gpu()
    X = synth.svd_matrix(5000, 6, 1e3, 7)
    _, _, _, info = borth.orthonormalize(dev(X), gram=gram, fact="svqb", passes=2)
    assert info.status == 0 and info.svqb_lifted == 0
    X[:, 2] = 0.0
    Q, _, _, info = borth.orthonormalize(dev(X), gram=gram, fact="svqb", passes=2)
    note("svqb lift, zero column", gram, info)
    assert info.status == 0 and info.svqb_lifted == 1
    Qh = Q.cpu().numpy()
    assert np.isfinite(Qh).all() and not Qh[:, 2].any()
