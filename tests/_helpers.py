"""Small matrix builders shared by the tests (no solver arithmetic)."""
import numpy as np
import scipy.sparse as sp

from paper_2009_12101_amd import problems as P

# The oracle variant that computes steps 5-10 as the library does by default
# (the Gram-form re-dot and the one-pass update); GPU parity tests of the
# default path compare against it.  The oracle's own default is Fig. 1 as
# written, which the full-size error test and the explicit-re-dot variant
# tests keep as their reference.
LIB_DEFAULT = ("gram", "onepass")


def csr_from_dense(M, name="dense"):
    S = sp.csr_matrix(M)
    S.sort_indices()
    return P.CSR(M.shape[0], S.indptr.astype(np.int32), S.indices.astype(np.int32),
                 S.data.astype(np.float64), name=name)


def csr_from_scipy(S, name="scipy"):
    S = sp.csr_matrix(S)
    S.sort_indices()
    return P.CSR(S.shape[0], S.indptr.astype(np.int32), S.indices.astype(np.int32),
                 S.data.astype(np.float64), name=name)
