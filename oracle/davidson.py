"""Davidson's method for the lowest eigenpair of the effective two-site problem (Eq. h_mat).

The paper names the method (Sections 2.1 and 2.2.1) but not its details; this oracle fixes them:

* start from the given guess, normalised;
* subspace V (orthonormal), W = H V; Rayleigh matrix G = sym(V^T W); lowest Ritz pair (theta, s);
* u = V s, residual r = W s - theta u; stop when ||r||_2 <= tol;
* correction t_i = r_i / (theta - D_i) with D = diag(H) and |theta - D_i| floored at 1e-8
  (sign kept); classical Gram-Schmidt applied twice against V, normalise, append;
* when V reaches ``max_sub`` vectors, restart with span{u, previous u} (orthonormalised).
"""
import numpy as np


def davidson(apply_h, diag, guess, tol=1e-10, max_iter=500, max_sub=24, precond=None):
    """Return dict(energy, vector, resid, iters, matvecs, converged, history)."""
    v = guess / np.linalg.norm(guess)
    V = [v]
    W = [apply_h(v)]
    matvecs = 1
    u_prev = None
    history = []
    theta, u, rnorm = None, v, np.inf
    for it in range(1, max_iter + 1):
        Vm = np.stack(V, axis=1)
        Wm = np.stack(W, axis=1)
        G = Vm.T @ Wm
        G = 0.5 * (G + G.T)
        evals, evecs = np.linalg.eigh(G)
        theta = evals[0]
        s = evecs[:, 0]
        u = Vm @ s
        r = Wm @ s - theta * u
        rnorm = np.linalg.norm(r)
        history.append((theta, rnorm))
        if rnorm <= tol:
            return dict(energy=theta, vector=u, resid=rnorm, iters=it, matvecs=matvecs,
                        converged=True, history=history)
        if precond is None:
            den = theta - diag
            den = np.where(np.abs(den) < 1e-8, np.where(den < 0, -1e-8, 1e-8), den)
            t = r / den
        else:
            t = precond(r, theta, u)
        if len(V) >= max_sub:
            basis = [u] if u_prev is None else [u, u_prev]
            V, W = [], []
            for b in basis:
                for q in V:
                    b = b - (q @ b) * q
                for q in V:
                    b = b - (q @ b) * q
                nb = np.linalg.norm(b)
                if nb > 1e-12:
                    b = b / nb
                    V.append(b)
                    W.append(apply_h(b))
                    matvecs += 1
        for _ in range(2):
            for q in V:
                t = t - (q @ t) * q
        nt = np.linalg.norm(t)
        if nt < 1e-14:
            break
        t = t / nt
        V.append(t)
        W.append(apply_h(t))
        matvecs += 1
        u_prev = u
    return dict(energy=theta, vector=u, resid=rnorm, iters=it, matvecs=matvecs,
                converged=False, history=history)
