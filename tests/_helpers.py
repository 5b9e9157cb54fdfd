"""Small dense/sparse helpers for the oracle pins (fp64 numpy / scipy only)."""
import numpy as np
import scipy.sparse as sp


def dense(A):
    return sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n)).toarray()


def scaled_dense(A):
    D = dense(A)
    s = 1.0 / np.sqrt(np.abs(np.diag(D)))
    return s[:, None] * D * s[None, :], s


def csr_dense(rp, ci, v, n):
    return sp.csr_matrix((v, ci, rp), shape=(n, n)).toarray()


def random_sparse_system(n, density, seed, spd=False, diag_boost=1.5):
    """Random sparse matrix with a full diagonal, sorted CSR, for pins."""
    from workloads.matrices import CSR
    rs = np.random.default_rng(seed)
    M = sp.random(n, n, density=density, random_state=rs, format="csr")
    M.data = rs.standard_normal(M.data.size)
    if spd:
        M = M + M.T
    M = M.tolil()
    rowsum = np.abs(M.toarray()).sum(axis=1)
    for i in range(n):
        M[i, i] = diag_boost * rowsum[i] + 1.0
    M = M.tocsr()
    M.sort_indices()
    return CSR(n, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64), f"rand{n}")
