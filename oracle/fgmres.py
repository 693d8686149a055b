"""Right-preconditioned restarted flexible GMRES (test infrastructure).

Follows Sec. 3 (Krylov subspaces; GMRES and its restarted form GMRES(m)) and
Sec. 4 (right preconditioning A M^{-1} x^ = b, whose residual is the true
residual; a matrix-free M^{-1}).  The flexible variant (Saad, SIAM J. Sci.
Comput. 14, 1993) stores the preconditioned vectors z_j = M^{-1} v_j and
updates x with them, which allows a preconditioner that changes between
applications.  Settings of Sec. 6: zero initial iterate, stop when the
relative residual is below the tolerance.

Orthogonalisation is classical Gram-Schmidt applied twice (CGS2); the
Hessenberg least-squares problem is reduced with complex Givens rotations.
A cycle ends when the estimated residual |g_{j+1}| reaches rtol * ||b||, when
m steps are done, or on breakdown; the true residual ||b - A x|| / ||b|| is
then computed and decides convergence.
"""

import numpy as np


def fgmres(matvec, precond, b, x0=None, restart=30, rtol=1e-6, maxit=5000):
    """Solve A x = b.  Returns (x, info) with iterations, restarts, history."""
    b = np.asarray(b, dtype=np.complex128)
    n = b.shape[0]
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    info = {"iters": 0, "restarts": 0, "converged": False, "history": [], "rel_res": 0.0}
    if bnorm == 0.0:
        x[:] = 0
        info["converged"] = True
        return x, info
    m = restart
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        info["rel_res"] = beta / bnorm
        if beta <= rtol * bnorm:
            info["converged"] = True
            return x, info
        if info["iters"] >= maxit or not np.isfinite(beta):
            return x, info
        V = np.zeros((n, m + 1), dtype=np.complex128)
        Z = np.zeros((n, m), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        V[:, 0] = r / beta
        g[0] = beta
        jj = 0
        for j in range(m):
            Z[:, j] = precond(V[:, j])
            w = matvec(Z[:, j])
            h = np.zeros(j + 2, dtype=np.complex128)
            for _ in range(2):  # CGS2
                c = V[:, :j + 1].conj().T @ w
                w = w - V[:, :j + 1] @ c
                h[:j + 1] += c
            h[j + 1] = np.linalg.norm(w)
            # previous rotations
            for i in range(j):
                a, bb = h[i], h[i + 1]
                h[i] = cs[i] * a + sn[i] * bb
                h[i + 1] = -np.conj(sn[i]) * a + cs[i] * bb
            a, bb = h[j], h[j + 1]
            rho = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            if abs(a) == 0.0:
                cs[j], sn[j] = 0.0, 1.0
            else:
                cs[j] = abs(a) / rho
                sn[j] = (a / abs(a)) * np.conj(bb) / rho
            h[j] = cs[j] * a + sn[j] * bb
            h[j + 1] = 0.0
            H[:j + 2, j] = h
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            info["iters"] += 1
            jj = j + 1
            est = abs(g[j + 1]) / bnorm
            info["history"].append(est)
            breakdown = np.linalg.norm(w) == 0.0
            if not breakdown:
                V[:, j + 1] = w / np.linalg.norm(w)
            if breakdown or est <= rtol or info["iters"] >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:jj, :jj]), g[:jj])
        x = x + Z[:, :jj] @ y
        info["restarts"] += 1
