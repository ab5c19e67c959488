"""Kohn-Sham ground state used as the input active space (oracle; test
infrastructure only).

Algorithm 1 starts from ground-state orbitals and H_KS (ground-state block);
the paper obtains them with RMG's multigrid-preconditioned solver.  Here: a
self-consistent field loop on rho = sum_{i <= N_occ} 2 psi_i^2 with Pulay (DIIS)
density mixing, each fixed-potential eigenproblem solved by a block
preconditioned eigensolver (locally optimal block iteration with dense
Rayleigh-Ritz, preconditioned by the inverse of the FD kinetic dispersion plus a
shift).  On tiny grids the dense Hamiltonian is diagonalised directly instead.
The orbitals are returned h^3-orthonormal with a fixed sign convention (largest
component positive).
"""

import warnings

import numpy as np
from scipy.sparse.linalg import LinearOperator, lobpcg

from .grid import fd_coefficients_float, laplacian
from .hamiltonian import electrostatic, lda_x
from .system import v_ion, projectors, apply_vnl


def _kinetic_dispersion(sys, coeffs):
    nx, ny, nz = sys.n
    h = sys.h
    lam = 0.0
    out = np.zeros((nz, ny, nx))
    for ax, n in zip((2, 1, 0), (nx, ny, nz)):
        k = 2 * np.pi * np.fft.fftfreq(n, d=h)
        l1 = coeffs[0] + 2.0 * sum(coeffs[j] * np.cos(j * k * h) for j in range(1, len(coeffs)))
        shape = [1, 1, 1]
        shape[ax] = n
        out = out + (l1 / (h * h)).reshape(shape)
    del lam
    return -0.5 * out  # kinetic energy of each plane wave (>= 0)


class _Op:
    def __init__(self, sys, vloc):
        self.sys = sys
        self.coeffs = fd_coefficients_float(4)
        self.vloc = vloc
        self.projs = projectors(sys)
        self.kin = _kinetic_dispersion(sys, self.coeffs)

    def apply(self, X):
        """H applied to the rows of X[m, Ng]."""
        nx, ny, nz = self.sys.n
        f = X.reshape(-1, nz, ny, nx)
        out = (-0.5 * laplacian(f, self.sys.h, self.coeffs)).reshape(X.shape) + self.vloc[None, :] * X
        if self.projs:
            out += apply_vnl(X, self.projs, self.sys.h)
        return out

    def precond(self, R, shift):
        nx, ny, nz = self.sys.n
        f = np.fft.fftn(R.reshape(-1, nz, ny, nx), axes=(1, 2, 3))
        f /= (self.kin + shift)[None]
        return np.fft.ifftn(f, axes=(1, 2, 3)).real.reshape(R.shape)


def _orth(V):
    q, r = np.linalg.qr(V.T)
    keep = np.abs(np.diag(r)) > 1e-10 * np.max(np.abs(np.diag(r)))
    return q[:, keep].T


def eigensolve(op, X0, n_want, tol, max_iter=400, n_guard=8):
    """Lowest n_want eigenpairs of op by SciPy's LOBPCG with the kinetic
    preconditioner; the block carries n_guard extra vectors.  Finishes with a
    Rayleigh-Ritz rotation.  Returns (eigenvalues, vectors[n_want, Ng]
    Euclidean-orthonormal, max residual of the wanted pairs)."""
    nb = n_want + n_guard
    X = X0
    if X.shape[0] < nb:
        rng = np.random.default_rng(7)
        X = np.vstack([X, op.precond(rng.standard_normal((nb - X.shape[0], X.shape[1])), 2.0)])
    X = _orth(X[:nb])
    ng = X.shape[1]
    HX = op.apply(X)
    w0 = np.linalg.eigvalsh(0.5 * (X @ HX.T + HX @ X.T))
    shift = 0.5 - min(0.0, float(w0[0]))
    A = LinearOperator((ng, ng), matvec=lambda v: op.apply(v.reshape(1, -1)).ravel(),
                       matmat=lambda V: op.apply(np.ascontiguousarray(V.T)).T, dtype=np.float64)
    M = LinearOperator((ng, ng), matvec=lambda v: op.precond(v.reshape(1, -1), shift).ravel(),
                       matmat=lambda V: op.precond(np.ascontiguousarray(V.T), shift).T, dtype=np.float64)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        w, V = lobpcg(A, np.ascontiguousarray(X.T), M=M, tol=tol, maxiter=max_iter, largest=False)
    X = _orth(V.T)
    HX = op.apply(X)
    Hs = X @ HX.T
    w, c = np.linalg.eigh(0.5 * (Hs + Hs.T))
    X = c.T @ X
    HX = c.T @ HX
    res = float(np.max(np.linalg.norm(HX - w[:, None] * X, axis=1)[:n_want]))
    return w[:n_want], X[:n_want], res


def _fix_signs(X):
    i = np.argmax(np.abs(X), axis=1)
    s = np.sign(X[np.arange(X.shape[0]), i])
    return X * s[:, None]


def ground_state(sys, n_extra: int = 4, tol_rho: float = 1e-11, tol_res: float = 1e-10,
                 max_scf: int = 200, seed: int = 12345, verbose: bool = False):
    """Self-consistent LDA-exchange ground state of sys.

    Returns dict(psi[N, Ng] h^3-orthonormal, eps[N + n_extra], rho, scf_iters,
    rho_err, res)."""
    N = sys.n_orb
    nb = N + n_extra
    dv = sys.h ** 3
    vion = v_ion(sys).ravel()
    rng = np.random.default_rng(seed)
    nx, ny, nz = sys.n
    # smooth random start vectors
    X = rng.standard_normal((nb, sys.ng))
    op = _Op(sys, vion)
    X = op.precond(X, 2.0)
    w, X, _ = eigensolve(op, X, nb, 1e-4)
    rho = 2.0 * np.sum(X[: sys.n_occ] ** 2, axis=0) / dv
    hist_in, hist_res = [], []
    err = np.inf
    it = 0
    for it in range(1, max_scf + 1):
        vh, _ = electrostatic(rho, sys)
        vx, _ = lda_x(rho)
        op = _Op(sys, vion + vh + vx)
        etol = max(tol_res * np.sqrt(dv) * 0.1, min(1e-4, 0.01 * err))
        w, X, res = eigensolve(op, X, nb, etol)
        rho_out = 2.0 * np.sum(X[: sys.n_occ] ** 2, axis=0) / dv
        R = rho_out - rho
        err = float(np.max(np.abs(R)))
        if verbose:
            print(f"scf {it}: rho err {err:.3e}  eig res {res:.2e}  eps_homo {w[sys.n_occ-1]:.6f}", flush=True)
        if err < tol_rho:
            break
        hist_in.append(rho.copy())
        hist_res.append(R.copy())
        if len(hist_in) > 8:
            hist_in.pop(0)
            hist_res.pop(0)
        m = len(hist_in)
        A = np.array([[np.dot(hist_res[i], hist_res[j]) for j in range(m)] for i in range(m)])
        B = np.zeros((m + 1, m + 1))
        B[:m, :m] = A
        B[m, :m] = B[:m, m] = 1.0
        rhs = np.zeros(m + 1)
        rhs[m] = 1.0
        try:
            c = np.linalg.solve(B + 1e-30 * np.eye(m + 1), rhs)[:m]
        except np.linalg.LinAlgError:
            c = np.zeros(m)
            c[-1] = 1.0
        rho_opt = sum(ci * r for ci, r in zip(c, hist_in))
        res_opt = sum(ci * r for ci, r in zip(c, hist_res))
        rho = rho_opt + 0.3 * res_opt
    # final orbitals: eigenvectors of H[rho] with the converged input density
    vh, _ = electrostatic(rho, sys)
    vx, _ = lda_x(rho)
    op = _Op(sys, vion + vh + vx)
    w, X, res = eigensolve(op, X, nb, tol_res * np.sqrt(dv) * 0.1)
    X = _fix_signs(X)
    psi = X[:N] / np.sqrt(dv)
    rho_final = 2.0 * np.sum(psi[: sys.n_occ] ** 2, axis=0)
    return dict(psi=psi, eps=w, rho=rho_final, scf_iters=it,
                rho_err=float(np.max(np.abs(rho_final - rho))), res=res / np.sqrt(dv))


def dense_ground_state(sys, max_scf: int = 200, tol_rho: float = 1e-12):
    """Same self-consistent problem solved with dense diagonalisation of the
    full grid Hamiltonian (tiny grids only)."""
    dv = sys.h ** 3
    coeffs = fd_coefficients_float(4)
    nx, ny, nz = sys.n
    ng = sys.ng
    eye = np.eye(ng).reshape(ng, nz, ny, nx)
    T = (-0.5 * laplacian(eye, sys.h, coeffs)).reshape(ng, ng)
    projs = projectors(sys)
    Vnl = apply_vnl(np.eye(ng), projs, sys.h) if projs else 0.0
    vion = v_ion(sys).ravel()
    H0 = T + Vnl
    w, U = np.linalg.eigh(H0 + np.diag(vion))
    rho = 2.0 * np.sum(U[:, : sys.n_occ] ** 2, axis=1) / dv
    hist_in, hist_res = [], []
    for it in range(1, max_scf + 1):
        vh, _ = electrostatic(rho, sys)
        vx, _ = lda_x(rho)
        Hm = H0 + np.diag(vion + vh + vx)
        w, U = np.linalg.eigh(0.5 * (Hm + Hm.T))
        rho_out = 2.0 * np.sum(U[:, : sys.n_occ] ** 2, axis=1) / dv
        R = rho_out - rho
        if np.max(np.abs(R)) < tol_rho:
            break
        hist_in.append(rho.copy())
        hist_res.append(R.copy())
        if len(hist_in) > 8:
            hist_in.pop(0)
            hist_res.pop(0)
        m = len(hist_in)
        B = np.zeros((m + 1, m + 1))
        for i in range(m):
            for j in range(m):
                B[i, j] = np.dot(hist_res[i], hist_res[j])
        B[m, :m] = B[:m, m] = 1.0
        rhs = np.zeros(m + 1)
        rhs[m] = 1.0
        c = np.linalg.solve(B, rhs)[:m]
        rho = sum(ci * r for ci, r in zip(c, hist_in)) + 0.3 * sum(ci * r for ci, r in zip(c, hist_res))
    vh, _ = electrostatic(rho, sys)
    vx, _ = lda_x(rho)
    Hm = H0 + np.diag(vion + vh + vx)
    w, U = np.linalg.eigh(0.5 * (Hm + Hm.T))
    X = _fix_signs(U.T)
    return dict(eps=w, psi_all=X / np.sqrt(dv), rho=rho, H_grid=Hm, scf_iters=it)
