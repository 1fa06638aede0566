"""Landau-Lifshitz frame (Sec. II.A, eqs. landau-lifshitz-first/second-moment).

eps U^alpha = T^{alpha beta} U_beta,  n = U_alpha N^alpha,  U.U = 1.
The oracle solves the eigenvalue problem directly: with the Minkowski metric
eta = diag(1, -1, -1, -1), T^{alpha beta} U_beta = (T eta) U, so U is the
eigenvector of the mixed tensor T eta whose direction is timelike (U.U > 0),
normalised to U.U = 1 with U^0 > 0, and eps is its eigenvalue (the other
eigenvalues belong to spacelike eigenvectors).
"""
import numpy as np


def landau_frame(Tmn, Nmu):
    """Tmn: [S, d, d] symmetric contravariant energy-momentum tensor (d = 3 for
    (t, x, y) or 4 for (t, x, y, z)), Nmu: [S, d].  Returns eps [S], U [S, d]
    (contravariant), n [S]."""
    d = Tmn.shape[-1]
    eta = np.diag([1.0] + [-1.0] * (d - 1))
    M = Tmn @ eta
    w, V = np.linalg.eig(M)
    w = w.real
    V = V.real
    norm = np.einsum("sik,ij,sjk->sk", V, eta, V)          # U.U of each eigenvector
    k = np.argmax(norm, axis=1)                             # the timelike one
    S = np.arange(Tmn.shape[0])
    U = V[S, :, k]
    U = U / np.sqrt(norm[S, k])[:, None]
    U = U * np.sign(U[:, :1])
    eps = w[S, k]
    n = np.einsum("si,ij,sj->s", U, eta, Nmu)
    return eps, U, n
