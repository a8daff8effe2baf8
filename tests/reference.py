"""Reference solutions U^E = A^{-1} F of the oracle's operator for the GPU
parity tests.

The plain definition of what the solver reaches is the exact discrete
solution of the upwind 5-point system (Sec. 3).  Where the oracle's own
FGMRES is slow (hundreds of restarted iterations at eps near 1e-2 or 5e-4,
where the preconditioner is weak), the reference is a sparse direct solve
(SuperLU, a library routine) of the oracle's assembled matrix, with its
Jacobi-scaled residual checked.  Nothing here touches the HIP path.
"""
import numpy as np
import scipy.sparse.linalg as sla


def direct(op, F, transpose=False):
    """(u, scaled relative residual) of A u = F (or A^T u = F) by SuperLU on
    the oracle's CSR matrix."""
    A = op.csr()
    if transpose:
        A = A.T
    A = A.tocsc()
    lu = sla.splu(A, permc_spec="MMD_AT_PLUS_A")
    u = lu.solve(np.ascontiguousarray(F, dtype=np.float64))
    d = np.sqrt(A.diagonal())
    res = np.linalg.norm((F - A @ u) / d) / np.linalg.norm(F / d)
    return u, res


def max_rel(a, b):
    """max-norm difference of a and b relative to max |b|."""
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(b).max())
