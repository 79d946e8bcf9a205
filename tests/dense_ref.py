"""Dense linear-algebra references for small problems (tests only).

Everything here is written from the paper's definitions with numpy/scipy
matrices, independently of the oracle's sparse loops:
  * the MAP cost's normal equations for the quadratic prior (eq. (global_obj)),
    H = A^T Lambda A + L_b / sigma_x^2, with L_b the weighted graph Laplacian of
    the 8-neighbour cliques;
  * the per-agent Hessians H_i = A_i^T Lambda_i A_i + L_b / (N sigma_x^2) and
    b_i = A_i^T Lambda_i y_i (proof of Theorem 2, with Lambda in b_i);
  * the closed form of one raster ICD pass, eq. (ICDUpdate1);
  * the augmented linear map of partial-update MACE, eq. (PUCEupdate), for a
    quadratic problem (Theorem 2) -- built exactly, without the first-order
    approximation in sigma^2.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

B_EDGE = 1.0 / (4.0 + 2.0 * np.sqrt(2.0))
B_DIAG = 1.0 / (4.0 * np.sqrt(2.0) + 4.0)


def dense_A(g, col_ptr, row, val):
    return sp.csc_matrix((val.astype(np.float64), row, col_ptr),
                         shape=(g.n_rows, g.n)).toarray()


def laplacian(nx, ny, b_edge=B_EDGE, b_diag=B_DIAG):
    n = nx * ny
    L = np.zeros((n, n))
    for i in range(ny):
        for j in range(nx):
            s = i * nx + j
            for di in (-1, 0, 1):
                for dj in (-1, 0, 1):
                    if di == 0 and dj == 0:
                        continue
                    ii, jj = i + di, j + dj
                    if 0 <= ii < ny and 0 <= jj < nx:
                        b = b_diag if (di and dj) else b_edge
                        L[s, s] += b
                        L[s, ii * nx + jj] -= b
    return L


def agent_rows(g, view_agent, i):
    r = np.arange(g.n_rows)
    return np.where(np.asarray(view_agent)[r // g.n_channels] == i)[0]


def map_quadratic(A, lam, y, Lb, sigma_x):
    H = A.T @ (lam[:, None] * A) + Lb / sigma_x ** 2
    return sla.cho_solve(sla.cho_factor(H), A.T @ (lam * y))


def agent_system(g, A, lam, y, Lb, sigma_x, view_agent, N):
    Hs, bs = [], []
    for i in range(N):
        r = agent_rows(g, view_agent, i)
        Ai, li = A[r], lam[r]
        Hs.append(Ai.T @ (li[:, None] * Ai) + Lb / (N * sigma_x ** 2))
        bs.append(Ai.T @ (li * y[r]))
    return Hs, bs


def icd_pass_closed_form(H, b, x, v, sigma):
    """eq. (ICDUpdate1): -(L + D + sigma^-2 I)^-1 (L^T x - b - sigma^-2 v)."""
    L = np.tril(H, -1)
    D = np.diag(np.diag(H))
    n = H.shape[0]
    return -np.linalg.solve(L + D + np.eye(n) / sigma ** 2, L.T @ x - b - v / sigma ** 2)


def pu_mace_linear_map(Hs, bs, sigma, rho):
    """Exact (M, c) with [w; X]_{k+1} = M [w; X]_k + c (eq. (PUCEupdate))."""
    N = len(Hs)
    n = Hs[0].shape[0]
    Nn = N * n
    P = np.zeros((Nn, Nn))
    Q = np.zeros((Nn, Nn))
    c0 = np.zeros(Nn)
    for i, (H, b) in enumerate(zip(Hs, bs)):
        L = np.tril(H, -1)
        D = np.diag(np.diag(H))
        Minv = np.linalg.inv(L + D + np.eye(n) / sigma ** 2)
        sl = slice(i * n, (i + 1) * n)
        P[sl, sl] = -Minv @ L.T
        Q[sl, sl] = Minv / sigma ** 2
        c0[sl] = Minv @ b
    Gm = np.kron(np.ones((N, N)) / N, np.eye(n))
    R = 2 * Gm - np.eye(Nn)
    M = np.zeros((2 * Nn, 2 * Nn))
    M[Nn:, :Nn] = Q @ R
    M[Nn:, Nn:] = P
    M[:Nn, :Nn] = rho * (2 * Q @ R - R) + (1 - rho) * np.eye(Nn)
    M[:Nn, Nn:] = 2 * rho * P
    c = np.concatenate([2 * rho * c0, c0])
    return M, c


def sor_pass_closed_form(H, b, x, v, sigma, omega):
    """Successive over-relaxation sweep (textbook SOR) for
    (H + I/sigma^2) z = b + v/sigma^2 from z = x:
      (D + omega L) z = omega (b + v/sigma^2) - (omega L^T + (omega - 1) D) x
    with D the diagonal of H + I/sigma^2 and L the strict lower triangle of H."""
    n = H.shape[0]
    M = H + np.eye(n) / sigma ** 2
    L = np.tril(M, -1)
    D = np.diag(np.diag(M))
    rhs = omega * (b + v / sigma ** 2) - (omega * L.T + (omega - 1.0) * D) @ x
    return np.linalg.solve(D + omega * L, rhs)


def laplacian3(nx, ny, nz, b_axial, b_edge=B_EDGE, b_diag=B_DIAG):
    """Weighted graph Laplacian of a stack of nz slices: the 8-neighbour
    in-plane cliques of every slice and the axial cliques (z, s)-(z+1, s)
    with weight b_axial; voxel v = z * nx * ny + s."""
    n = nx * ny
    L = np.kron(np.eye(nz), laplacian(nx, ny, b_edge, b_diag))
    P = np.zeros((nz, nz))
    for z in range(nz - 1):
        P[z, z] += 1.0
        P[z + 1, z + 1] += 1.0
        P[z, z + 1] -= 1.0
        P[z + 1, z] -= 1.0
    return L + b_axial * np.kron(P, np.eye(n))


def volume_system(A, lam, y, nz):
    """Block-diagonal data Hessian and right side of a slice stack measured
    by one 2-D matrix A: H_data = blockdiag(A^T Lambda_z A), b = A^T Lambda_z y_z."""
    m, n = A.shape
    H = np.zeros((nz * n, nz * n))
    b = np.zeros(nz * n)
    for z in range(nz):
        lz, yz = lam[z * m:(z + 1) * m], y[z * m:(z + 1) * m]
        H[z * n:(z + 1) * n, z * n:(z + 1) * n] = A.T @ (lz[:, None] * A)
        b[z * n:(z + 1) * n] = A.T @ (lz * yz)
    return H, b
