"""Restarted GMRES (the solver of paper Sec. III-A, tolerance and restart per Sec. IV-C).

Reading: zero initial guess, classical Gram-Schmidt applied twice (CGS2) in FP64, unpreconditioned
relative residual ||b - A x|| / ||b||, Givens rotations on the Hessenberg matrix, restart m.

Parity pins (tests): on small random systems it reaches the requested residual and agrees with
a dense direct solve; with restart >= n it terminates in at most n iterations.
"""
import numpy as np


def gmres(matvec, b, tol=1e-6, restart=50, max_iter=1000):
    """Returns (x, iterations, relative residual history of the Arnoldi estimate)."""
    b = np.asarray(b, np.complex128)
    n = len(b)
    x = np.zeros(n, np.complex128)
    bnorm = np.linalg.norm(b)
    if bnorm == 0:
        return x, 0, [0.0]
    hist = [1.0]
    it = 0
    while it < max_iter:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            break
        V = np.zeros((restart + 1, n), np.complex128)
        H = np.zeros((restart + 1, restart), np.complex128)
        cs = np.zeros(restart, np.complex128)
        sn = np.zeros(restart, np.complex128)
        g = np.zeros(restart + 1, np.complex128)
        g[0] = beta
        V[0] = r / beta
        j_end = 0
        for j in range(restart):
            w = matvec(V[j])
            h = V[:j + 1].conj() @ w
            w = w - h @ V[:j + 1]
            h2 = V[:j + 1].conj() @ w
            w = w - h2 @ V[:j + 1]
            H[:j + 1, j] = h + h2
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = np.conj(cs[i]) * H[i, j] + np.conj(sn[i]) * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            cs[j] = a / den if den > 0 else 1.0
            sn[j] = bb / den if den > 0 else 0.0
            H[j, j] = cs[j].conj() * a + sn[j].conj() * bb
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            it += 1
            j_end = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) / bnorm <= tol or it >= max_iter:
                break
        y = np.linalg.solve(np.triu(H[:j_end, :j_end]), g[:j_end])
        x = x + y @ V[:j_end]
        if hist[-1] <= tol:
            r = b - matvec(x)
            if np.linalg.norm(r) / bnorm <= tol:
                break
    return x, it, hist
