"""Krylov solvers in the M inner product (oracle; test infrastructure only).

Sec. 4.5: M A_h is symmetric (each term of the polynomial M P(M^-1 W) is),
and A_h is positive definite with eigenvalues in (0, 3/2) (Sec. 3), so CG
applies to M(I - S_h) u = M b (eq. (amat_sym)).

Reading of eq. (amat_sym): CG is run on A_h in the M inner product
(x, y)_M = sum_i m_i x_i y_i.  It minimises the same M A_h-norm of the error
as CG on the matrix M A_h would, its Krylov space is K(A_h, b), and its
eigenvalues are those of A_h.  The two coincide when M is a multiple of the
identity (constant rho, all-Dirichlet).  The stopping test is
||r||_M <= tol ||b||_M; the paper measures residuals relative to the
zero-guess residual, which is b.

Conjugate residual (the Remark at the end of Sec. 4.5), MINRES (the remedy
the remark in Sec. 4.4 recommends when A_h is slightly indefinite near
resonance) and restarted GMRES (used for non-symmetric problems in Sec. 5.4)
are provided in the same inner product.
"""

import math

import numpy as np


class KrylovResult:
    def __init__(self, x, iters, converged, history, alphas=None, betas=None):
        self.x = x
        self.iters = iters
        self.converged = converged
        self.history = history        # ||r_k||_M / ||b||_M, k = 0..iters
        self.alphas = alphas or []
        self.betas = betas or []

    def lanczos_cond(self):
        """Condition estimate from the CG coefficients (the Lanczos tridiagonal)."""
        a, b = self.alphas, self.betas
        k = len(a)
        if k == 0:
            return float("nan")
        T = np.zeros((k, k))
        for i in range(k):
            T[i, i] = 1.0 / a[i] + (b[i - 1] / a[i - 1] if i > 0 else 0.0)
            if i + 1 < k:
                T[i, i + 1] = T[i + 1, i] = math.sqrt(b[i]) / a[i]
        ev = np.linalg.eigvalsh(T)
        return float(ev[-1] / ev[0])


def _mdot(m, x, y):
    return float(np.dot(m * x, y))


def cg(apply_A, b, m, x0=None, tol=1e-10, maxit=1000):
    """Conjugate gradients on A in the M inner product."""
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, np.float64).copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    p = r.copy()
    rr = _mdot(m, r, r)
    bn = math.sqrt(_mdot(m, b, b))
    hist = [math.sqrt(rr) / bn]
    alphas, betas = [], []
    if hist[-1] <= tol:
        return KrylovResult(x, 0, True, hist, alphas, betas)
    for k in range(1, maxit + 1):
        q = apply_A(p)
        pq = _mdot(m, p, q)
        if not pq > 0:
            raise ArithmeticError("CG breakdown: (p, A p)_M <= 0")
        alpha = rr / pq
        x += alpha * p
        r -= alpha * q
        rr_new = _mdot(m, r, r)
        hist.append(math.sqrt(rr_new) / bn)
        alphas.append(alpha)
        if hist[-1] <= tol:
            return KrylovResult(x, k, True, hist, alphas, betas)
        beta = rr_new / rr
        betas.append(beta)
        p = r + beta * p
        rr = rr_new
    return KrylovResult(x, maxit, False, hist, alphas, betas)


def cr(apply_A, b, m, x0=None, tol=1e-10, maxit=1000):
    """Conjugate residual on A in the M inner product (A M-self-adjoint)."""
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, np.float64).copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    bn = math.sqrt(_mdot(m, b, b))
    hist = [math.sqrt(_mdot(m, r, r)) / bn]
    if hist[-1] <= tol:
        return KrylovResult(x, 0, True, hist)
    p = r.copy()
    Ar = apply_A(r)
    Ap = Ar.copy()
    rAr = _mdot(m, r, Ar)
    for k in range(1, maxit + 1):
        alpha = rAr / _mdot(m, Ap, Ap)
        x += alpha * p
        r -= alpha * Ap
        hist.append(math.sqrt(_mdot(m, r, r)) / bn)
        if hist[-1] <= tol:
            return KrylovResult(x, k, True, hist)
        Ar = apply_A(r)
        rAr_new = _mdot(m, r, Ar)
        beta = rAr_new / rAr
        p = r + beta * p
        Ap = Ar + beta * Ap
        rAr = rAr_new
    return KrylovResult(x, maxit, False, hist)


def gmres(apply_A, b, m, x0=None, tol=1e-10, maxit=1000, restart=30):
    """Restarted GMRES with classical Gram-Schmidt applied twice, in the M
    inner product; least squares by Givens rotations."""
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, np.float64).copy()
    bn = math.sqrt(_mdot(m, b, b))
    hist = []
    total = 0
    while True:
        r = b - apply_A(x) if (x0 is not None or total > 0) else b.copy()
        beta = math.sqrt(_mdot(m, r, r))
        hist.append(beta / bn)
        if beta / bn <= tol or total >= maxit:
            return KrylovResult(x, total, beta / bn <= tol, hist)
        V = [r / beta]
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        j_done = 0
        for j in range(restart):
            w = apply_A(V[j])
            total += 1
            for _ in range(2):                       # CGS2
                Vm = np.array(V)
                coeff = Vm @ (m * w)
                w = w - Vm.T @ coeff
                H[: j + 1, j] += coeff
            hn = math.sqrt(_mdot(m, w, w))
            H[j + 1, j] = hn
            for i in range(j):                        # apply old rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rho_ = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / rho_, H[j + 1, j] / rho_
            H[j, j] = rho_
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            j_done = j + 1
            hist.append(abs(g[j + 1]) / bn)
            if abs(g[j + 1]) / bn <= tol or total >= maxit or hn == 0.0:
                break
            V.append(w / hn)
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        x = x + np.array(V[:j_done]).T @ y


def minres(apply_A, b, m, x0=None, tol=1e-10, maxit=1000):
    """MINRES on an M-self-adjoint A in the M inner product (the remark in
    Sec. 4.4 recommends it when A_h is indefinite near resonance).

    Written from its definition (Paige and Saunders, 1975): x_k minimises
    ||b - A x||_M over x0 + K_k(A, r0).  The Lanczos process in the M inner
    product gives A V_k = V_{k+1} Tbar_k with M-orthonormal V and the
    (k+1) x k tridiagonal Tbar_k (diagonal alpha_j, off-diagonals beta_{j+1}),
    so ||r_k||_M = min_y ||beta_1 e_1 - Tbar_k y||_2.  That small least-squares
    problem is solved by a QR factorisation of Tbar_k built one Givens rotation
    per column; x_k = x_0 + V_k R_k^{-1} t_k is updated through the direction
    vectors D_k = V_k R_k^{-1}, and |last entry of the rotated right-hand side|
    is ||r_k||_M.
    """
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, np.float64).copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    bn = math.sqrt(_mdot(m, b, b))
    beta = math.sqrt(_mdot(m, r, r))          # beta_1
    hist = [beta / bn]
    if hist[-1] <= tol:
        return KrylovResult(x, 0, True, hist)
    v_prev = np.zeros_like(b)
    v = r / beta
    d_prev2 = np.zeros_like(b)                # d_{j-2}
    d_prev = np.zeros_like(b)                 # d_{j-1}
    c2, s2 = 1.0, 0.0                         # rotation G_{j-2}
    c1, s1 = 1.0, 0.0                         # rotation G_{j-1}
    g = beta                                  # j-th entry of the rotated rhs, before G_j
    for k in range(1, maxit + 1):
        # Lanczos: beta_{j+1} v_{j+1} = A v_j - alpha_j v_j - beta_j v_{j-1}
        q = apply_A(v)
        alpha = _mdot(m, v, q)
        q = q - alpha * v - beta * v_prev
        beta_next = math.sqrt(_mdot(m, q, q))
        # column j of Tbar: (beta_j, alpha_j, beta_{j+1}) in rows j-1, j, j+1;
        # apply G_{j-2} (rows j-2, j-1) then G_{j-1} (rows j-1, j)
        b_j = beta if k > 1 else 0.0          # Tbar has no entry above its first diagonal
        eps = s2 * b_j
        t = c2 * b_j
        delta = c1 * t + s1 * alpha
        gbar = -s1 * t + c1 * alpha
        # new rotation G_j zeroes beta_{j+1}
        gamma = math.hypot(gbar, beta_next)
        if gamma == 0.0:
            raise ArithmeticError("MINRES breakdown: singular tridiagonal")
        c, s = gbar / gamma, beta_next / gamma
        tau = c * g
        g = -s * g
        # d_j = (v_j - delta d_{j-1} - eps d_{j-2}) / gamma;  x_j = x_{j-1} + tau d_j
        d = (v - delta * d_prev - eps * d_prev2) / gamma
        x += tau * d
        hist.append(abs(g) / bn)
        if hist[-1] <= tol or beta_next == 0.0:
            return KrylovResult(x, k, True, hist)
        d_prev2, d_prev = d_prev, d
        c2, s2, c1, s1 = c1, s1, c, s
        v_prev, v = v, q / beta_next
        beta = beta_next
    return KrylovResult(x, maxit, False, hist)
