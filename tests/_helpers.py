"""Small matrix builders shared by the tests (no solver arithmetic)."""
import numpy as np
import scipy.sparse as sp

from paper_2009_12101_amd import problems as P

# GPU parity tests of the library's default path compare against the
# oracle's default, Fig. 1 as written (FIG1: no variant).  The oracle's
# ("gram", "onepass") variant restates the library's default arrangement of
# steps 5-10 (Gram-form re-dot, one update); tests that use it are labelled
# cross-checks of that arrangement, not parity with the paper.
FIG1 = ()
ONEPASS_CROSSCHECK = ("gram", "onepass")


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
