"""Independent matrix construction of fermion operators (tests only).

Jordan-Wigner: with M spin-orbitals, a_j = I x ... x I x s- x Z x ... x Z
(Kronecker factors ordered from mode M-1 down to mode 0, so that basis index
bit j is the occupation of mode j; Z = diag(1, -1), s- = [[0, 1], [0, 0]]).
Spin-orbital order follows the paper's string x = (sigma_alpha, sigma_beta)
(Sec. 2.1): alpha orbitals are modes 0..norb-1, beta orbitals norb..2norb-1.
Everything here is matrix algebra on the Fock space and shares nothing with
the bit-string code of the oracle or of the GPU library.
"""
import numpy as np
import scipy.sparse as sp

_Z = sp.csr_matrix(np.diag([1.0, -1.0]))
_I = sp.identity(2, format="csr")
_SM = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]]))


def annihilators(nmodes):
    ops = []
    for j in range(nmodes):
        m = None
        for mode in range(nmodes - 1, -1, -1):
            f = _SM if mode == j else (_Z if mode < j else _I)
            m = f if m is None else sp.kron(m, f, format="csr")
        ops.append(m.tocsr())
    return ops


def hamiltonian(h, eri, e_core):
    """Full Fock-space H = E_core + sum h_PQ a+_P a_Q + 1/2 sum (pr|qs) a+_P a+_Q a_S a_R."""
    norb = h.shape[0]
    M = 2 * norb
    a = annihilators(M)
    ad = [x.T.tocsr() for x in a]
    dim = 2 ** M
    H = sp.identity(dim, format="csr") * e_core
    spin = [0] * norb + [1] * norb
    E = {}
    for P in range(M):
        for R in range(M):
            if spin[P] == spin[R]:
                E[P, R] = (ad[P] @ a[R]).tocsr()
    for P in range(M):
        for Q in range(M):
            if spin[P] == spin[Q]:
                H = H + h[P % norb, Q % norb] * E[P, Q]
    # a+_P a+_Q a_S a_R = E_PR E_QS - delta_QR E_PS
    for P in range(M):
        for R in range(M):
            if spin[P] != spin[R]:
                continue
            for Q in range(M):
                for S in range(M):
                    if spin[Q] != spin[S]:
                        continue
                    g = eri[P % norb, R % norb, Q % norb, S % norb]
                    if g == 0.0:
                        continue
                    term = E[P, R] @ E[Q, S]
                    if Q == R:
                        term = term - E[P, S]
                    H = H + 0.5 * g * term
    return H.tocsr()


def basis_index(alpha, beta, norb):
    """Fock-space index of determinant (alpha, beta): bits alpha | beta << norb."""
    return (np.asarray(alpha, dtype=np.uint64) |
            (np.asarray(beta, dtype=np.uint64) << np.uint64(norb))).astype(np.int64)


def projected(h, eri, e_core, alpha, beta):
    """Dense H_B in the caller's determinant order via the Fock-space matrix."""
    norb = h.shape[0]
    H = hamiltonian(h, eri, e_core)
    idx = basis_index(alpha, beta, norb)
    return H[idx][:, idx].toarray()


def op_matrix_element(norb, xi, xj, creators, annihilators_):
    """<x_i| a+_{c0} a+_{c1} ... a_{a0} a_{a1} ... |x_j> with the operators applied
    right to left (annihilators_ listed left to right as written)."""
    M = 2 * norb
    a = annihilators(M)
    m = sp.identity(2 ** M, format="csr")
    for c in creators:
        m = m @ a[c].T
    for d in annihilators_:
        m = m @ a[d]
    return m[int(xi), int(xj)]
