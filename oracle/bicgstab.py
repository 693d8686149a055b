"""Right-preconditioned BiCGSTAB (test infrastructure).

Follows Sec. 3, which names the Bi-Conjugate Gradient Stabilized method (van
der Vorst, SIAM J. Sci. Stat. Comput. 13, 1992) as the short-recurrence
alternative to GMRES and compares the two with the FMM preconditioner.  The
iteration is van der Vorst's, applied to A M^{-1} y = b with x = M^{-1} y
(right preconditioning, Sec. 4, so the recursive residual is that of A x = b):

    r0 = b - A x0,  r^ = r0,  rho = alpha = omega = 1,  v = p = 0
    repeat:  rho_i = (r^, r);  beta = (rho_i / rho) (alpha / omega)
             p = r + beta (p - omega v);  p^ = M^{-1} p;  v = A p^
             alpha = rho_i / (r^, v);  s = r - alpha v
             s^ = M^{-1} s;  t = A s^;  omega = (t, s) / (t, t)
             x += alpha p^ + omega s^;  r = s - omega t

with (a, b) = conj(a).b.  It stops when ||r|| <= rtol ||b|| (then the true
residual is returned with x), after maxit iterations, or on breakdown (a zero
rho or (r^, v)).
"""

import numpy as np


def bicgstab(matvec, precond, b, x0=None, rtol=1e-6, maxit=5000):
    """Solve A x = b.  Returns (x, info) with iterations and the residual history."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    info = {"iters": 0, "converged": False, "history": [], "breakdown": False}
    if bnorm == 0.0:
        info["converged"] = True
        info["rel_res"] = 0.0
        return np.zeros_like(b), info
    r = b - matvec(x)
    rh = r.copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    while np.linalg.norm(r) > rtol * bnorm and info["iters"] < maxit:
        rho_i = np.vdot(rh, r)
        if info["iters"] == 0:
            beta = 0.0
        else:
            if rho == 0 or omega == 0:
                info["breakdown"] = True
                break
            beta = (rho_i / rho) * (alpha / omega)
        rho = rho_i
        p = r + beta * (p - omega * v)
        ph = precond(p)
        v = matvec(ph)
        d = np.vdot(rh, v)
        if d == 0:
            info["breakdown"] = True
            break
        alpha = rho / d
        s = r - alpha * v
        sh = precond(s)
        t = matvec(sh)
        tt = np.vdot(t, t)
        omega = np.vdot(t, s) / tt if tt != 0 else 0.0
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        info["iters"] += 1
        info["history"].append(np.linalg.norm(r) / bnorm)
    info["rel_res"] = np.linalg.norm(b - matvec(x)) / bnorm
    info["converged"] = bool(info["rel_res"] <= rtol)
    return x, info
