"""Solvers of the oracle (test infrastructure only).

The discrete problem (Sec. 2): find eps with
    A eps = b,   A = Id + Gamma0 * (C - C0)          (eq. (6))
    b = -Gamma0 * P_rhs                              (Algorithm 1 INIT; Sec. 3 for order >= 2)
where P_rhs = C:E for the classical problem and p_2 + theta_2 for the
strain-gradient problem.

Readings of the paper used here:
  * Basic Scheme: the fixed point of eq. (5), eps_{n+1} = b + eta_n with
    eta_n = -Gamma0 * ((C - C0) : eps_n), started at eps_0 = b.  (The update
    printed in Algorithm 1 would iterate eps_{n+1} = A eps_n, which diverges;
    Algorithm 1's body is the matrix-vector product of eq. (6).)
  * Stop rule: the Cauchy criterion ||eps_{n+1} - eps_n|| / ||eps_0|| < tol
    stated after Algorithm 1; the returned iterate is eps_{n+1} and the
    iteration count is n + 1.
  * CG: Hestenes-Stiefel conjugate gradients on eq. (6) in the C0 inner
    product <a, c> = sum_x (lam0 tr a tr c + 2 mu0 a : c), in which A is
    self-adjoint on compatible fields; start x_0 = b, stop when the
    recursive residual satisfies ||r||_L2 / ||b||_L2 < tol.
  * Zero right-hand side: if ||b|| <= 1e-14 * scale the solution is eps = 0
    after 0 iterations (the paper divides by ||eps_0||).
  * BiCGSTAB (the solver of the paper's experiments, Sec. 4): van der Vorst's
    method in the L2 inner product, x_0 = b, shadow residual r_0, the same
    stop rule as CG, checked once per iteration (two operator applications).
"""
import numpy as np

from . import spectral, tensors


class Problem:
    """Stiffness field + reference medium (Sec. 2)."""

    def __init__(self, cfield, lam0, mu0):
        if mu0 == 0.0 or lam0 + 2.0 * mu0 == 0.0:
            raise ValueError("reference medium must have mu0 != 0 and lam0 + 2 mu0 != 0")
        self.C = cfield
        self.lam0 = float(lam0)
        self.mu0 = float(mu0)
        self.C0 = tensors.isotropic_stiffness(lam0, mu0)
        self.shape = cfield.shape

    def green(self, tau):
        """-(Gamma0 * tau)."""
        return spectral.green_apply(tau, self.lam0, self.mu0)

    def polarization(self, eps):
        """(C - C0) : eps  (Algorithm 1, first step of the iteration)."""
        return self.C.contract(eps, minus=self.C0)

    def apply_A(self, eps):
        """(Id + Gamma0 * (C - C0)) : eps  (left-hand side of eq. (6))."""
        return eps - self.green(self.polarization(eps))

    def rhs(self, p_rhs):
        """b = -Gamma0 * P_rhs."""
        return self.green(p_rhs)

    def ip_c0(self, a, c):
        """C0 inner product sum_x (lam0 tr a tr c + 2 mu0 a : c)."""
        tra = np.einsum("ii...->...", a)
        trc = np.einsum("ii...->...", c)
        return float(self.lam0 * np.sum(tra * trc) + 2.0 * self.mu0 * np.sum(a * c))


def _guard(b, scale):
    return tensors.l2norm(b) <= 1e-14 * scale


def basic_scheme(prob, b, tol, max_iter=100000, scale=None):
    """Basic Scheme on A eps = b.  Returns (eps, info)."""
    nb = tensors.l2norm(b)
    history = []
    if scale is not None and _guard(b, scale):
        return np.zeros_like(b), {"iters": 0, "residual": 0.0, "history": history, "converged": True}
    eps = b.copy()
    for n in range(max_iter):
        eta = prob.green(prob.polarization(eps))
        eps_new = b + eta
        crit = tensors.l2norm(eps_new - eps) / nb
        history.append(crit)
        eps = eps_new
        if crit < tol:
            return eps, {"iters": n + 1, "residual": crit, "history": history, "converged": True}
    return eps, {"iters": max_iter, "residual": history[-1], "history": history, "converged": False}


def conjugate_gradient(prob, b, tol, max_iter=100000, scale=None):
    """CG on eq. (6) in the C0 inner product.  Returns (eps, info)."""
    nb = tensors.l2norm(b)
    history = []
    if scale is not None and _guard(b, scale):
        return np.zeros_like(b), {"iters": 0, "residual": 0.0, "history": history, "converged": True}
    x = b.copy()
    r = b - prob.apply_A(x)
    p = r.copy()
    rr = prob.ip_c0(r, r)
    for k in range(max_iter):
        q = prob.apply_A(p)
        alpha = rr / prob.ip_c0(p, q)
        x = x + alpha * p
        r = r - alpha * q
        crit = tensors.l2norm(r) / nb
        history.append(crit)
        if crit < tol:
            return x, {"iters": k + 1, "residual": crit, "history": history, "converged": True}
        rr_new = prob.ip_c0(r, r)
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, {"iters": max_iter, "residual": history[-1], "history": history, "converged": False}


def bicgstab(prob, b, tol, max_iter=100000, scale=None):
    """BiCGSTAB (van der Vorst's stabilised bi-conjugate gradients) on eq. (6),
    the Krylov solver the paper's experiments ran (Sec. 4).  A needs no
    symmetry here, so the plain L2 (Frobenius) inner product is used.  Start
    x_0 = b like the CG version, shadow residual r^ = r_0; one iteration is two
    operator applications and is checked after both.  Returns (eps, info)."""
    nb = tensors.l2norm(b)
    history = []
    if scale is not None and _guard(b, scale):
        return np.zeros_like(b), {"iters": 0, "residual": 0.0, "history": history, "converged": True}
    ip = tensors.frobenius
    x = b.copy()
    r = b - prob.apply_A(x)
    crit = tensors.l2norm(r) / nb
    if crit < tol:
        return x, {"iters": 0, "residual": crit, "history": history, "converged": True}
    r_hat = r.copy()
    rho_prev = alpha = omega = 1.0
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    for k in range(max_iter):
        rho = ip(r_hat, r)
        beta = (rho / rho_prev) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = prob.apply_A(p)
        alpha = rho / ip(r_hat, v)
        s = r - alpha * v
        t = prob.apply_A(s)
        omega = ip(t, s) / ip(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho_prev = rho
        crit = tensors.l2norm(r) / nb
        history.append(crit)
        if crit < tol:
            return x, {"iters": k + 1, "residual": crit, "history": history, "converged": True}
    return x, {"iters": max_iter, "residual": history[-1], "history": history, "converged": False}


def true_residual(prob, eps, b):
    """||b - A eps|| / ||b||  (the equilibrium residual)."""
    return tensors.l2norm(b - prob.apply_A(eps)) / tensors.l2norm(b)


# ---------------------------------------------------------------------------
# Dense displacement Galerkin solve: the definition of the discrete solution.
# ---------------------------------------------------------------------------

def _derivative_matrix_1d(n, with_derivative):
    """Real n x n matrix of the trigonometric derivative (or the Nyquist-free
    projection when with_derivative is False) built from explicit DFT matrices."""
    w = np.exp(-2j * np.pi * (np.outer(np.arange(n), np.arange(n)) % n) / n)   # forward
    winv = np.conj(w) / n
    j = np.arange(n)
    k = np.where(j < (n + 1) // 2, j, j - n).astype(np.float64)
    mask = np.ones(n)
    if n % 2 == 0:
        mask[k == -n // 2] = 0.0
    diag = (1j * 2.0 * np.pi * k * mask) if with_derivative else mask.astype(complex)
    m = winv @ np.diag(diag) @ w
    return np.real(m)


def dense_galerkin(cfield, e_macro=None, p_rhs=None):
    """Minimise sum_x (P + C:eps(u)) ... energy over trigonometric displacements.

    The unknown is the nodal displacement u (3 x n^3).  eps(u) = sym grad u with
    the trigonometric derivative on retained modes (eq. (1)).  For the
    classical problem the discrete energy is
        sum_x (E + eps(u)) : C(x) : (E + eps(u));
    for a polarization right-hand side P it is
        sum_x [ 1/2 eps(u) : C : eps(u) + P : eps(u) ].
    Both lead to the normal equations D^T C D u = -D^T f with f = C:E or P.
    Returns eps (3,3,n0,n1,n2).  Only for tiny grids (n^3 <= 125).
    """
    shape = cfield.shape
    nvox = int(np.prod(shape))
    mats = []
    for d in range(3):
        factors = [_derivative_matrix_1d(shape[e], with_derivative=(e == d)) for e in range(3)]
        mats.append(np.kron(np.kron(factors[0], factors[1]), factors[2]))    # C-order grid
    # D maps u (3, nvox) -> eps (3, 3, nvox)
    dmat = np.zeros((3, 3, nvox, 3, nvox))
    for i in range(3):
        for j in range(3):
            dmat[i, j, :, j, :] += 0.5 * mats[i]
            dmat[i, j, :, i, :] += 0.5 * mats[j]
    dmat = dmat.reshape(9 * nvox, 3 * nvox)
    # block-diagonal stiffness (9 nvox x 9 nvox)
    cmat = np.zeros((3, 3, nvox, 3, 3, nvox))
    flat = cfield.phase.ravel()
    for x in range(nvox):
        cmat[:, :, x, :, :, x] = cfield.tensors[flat[x]]
    cmat = cmat.reshape(9 * nvox, 9 * nvox)
    if p_rhs is None:
        f = cfield.contract_const(e_macro).reshape(9 * nvox)
    else:
        f = np.asarray(p_rhs).reshape(9 * nvox)
    k = dmat.T @ cmat @ dmat
    rhs = -dmat.T @ f
    u, *_ = np.linalg.lstsq(k, rhs, rcond=1e-12)
    return (dmat @ u).reshape((3, 3) + shape)
