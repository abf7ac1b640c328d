"""Order-0 and order-1 homogenization problems (test infrastructure only).

Naming: order 0 is the classical cell problem (the paper's alpha = 1,
polarization C:E and no body force, Sec. 3 Definition); order 1 is the
strain-gradient problem (alpha = 2) whose right-hand side is built from the
six order-0 correctors.

Unit loads: E^(J) is the engineering Voigt unit vector e_J, i.e. the tensor
e_k x e_k for J < 3 and (e_k x e_l + e_l x e_k)/2 for the shears.  With this
choice the order-0 displacement for E^(kl) is the corrector column X_1[., kl]
of the ansatz u_1 = X_1(y) : E(Y) (Sec. 3), and column J of the effective
stiffness is the Voigt vector of <sigma^(J)>.

Gradient load G[J, j] = d E_kl / d Y_j for the Voigt pair J = (k, l), tensor
components (not engineering).  Sums over symmetric pairs k <= l carry the
multiplicity c_J = 1 for J < 3 and 2 for the shears.
"""
import numpy as np

from . import fftref, solvers, spectral, tensors

MULT = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])


def make_problem(phase, lam0, mu0, lame=None, voigt21=None):
    if (lame is None) == (voigt21 is None):
        raise ValueError("give exactly one of lame / voigt21")
    cf = (tensors.StiffnessField.from_lame(phase, lame) if lame is not None
          else tensors.StiffnessField.from_voigt21(phase, voigt21))
    return solvers.Problem(cf, lam0, mu0)


def _solve(prob, p_rhs, scheme, tol, max_iter, scale):
    b = prob.rhs(p_rhs)
    if scheme == "basic":
        eps, info = solvers.basic_scheme(prob, b, tol, max_iter, scale=scale)
    elif scheme == "cg":
        eps, info = solvers.conjugate_gradient(prob, b, tol, max_iter, scale=scale)
    elif scheme == "bicgstab":
        eps, info = solvers.bicgstab(prob, b, tol, max_iter, scale=scale)
    else:
        raise ValueError(scheme)
    info["b_norm"] = tensors.l2norm(b)
    return eps, info


def guard_scale(p_rhs, mu0):
    """Strain-like scale ||C:E|| / (2 |mu0|) for the zero-right-hand-side guard of the
    classical problem; the strain-gradient problem uses (||p_2|| + ||g||) / (2 |mu0|)."""
    return tensors.l2norm(p_rhs) / (2.0 * abs(mu0))


def solve_order0(prob, e_voigt, scheme="cg", tol=1e-12, max_iter=100000):
    """Classical problem (alpha = 1): returns (eps (3,3,...), mean stress Voigt, info)."""
    e = tensors.tensor_from_engineering(e_voigt)
    p_rhs = prob.C.contract_const(e)                       # p_1 = C:E
    eps, info = _solve(prob, p_rhs, scheme, tol, max_iter, guard_scale(p_rhs, prob.mu0))
    sigma = prob.C.contract(eps + e[:, :, None, None, None])
    mean = tensors.stress_voigt_from_tensor(sigma.mean(axis=(2, 3, 4)))
    return eps, mean, info


def effective_stiffness(prob, scheme="cg", tol=1e-12, max_iter=100000):
    """6x6 Voigt C_eff from the six unit loads; also returns the six correctors."""
    ceff = np.zeros((6, 6))
    correctors = []
    infos = []
    for j in range(6):
        e = np.zeros(6)
        e[j] = 1.0
        eps, mean, info = solve_order0(prob, e, scheme, tol, max_iter)
        ceff[:, j] = mean
        correctors.append(eps)
        infos.append(info)
    return ceff, correctors, infos


def order1_rhs(prob, correctors, grad):
    """Right-hand side of the strain-gradient problem (alpha = 2, Sec. 3).

    correctors: six order-0 strain fields eps^(J) (3,3,...) for the unit loads.
    grad: (6, 3) array G[J, j] = dE_kl/dY_j.
    Returns (P = p_2 + theta_2 (3,3,...), p_2, theta_2, g (3,...), <g>).

      X_1[:, J]  displacement of corrector J (inverse of eq. (1))
      (X_1 . G)_mj = sum_J c_J X_1[m, J] G[J, j]
      p_2 = C : sym(X_1 . G)                                   (definition of p_2)
      S^(J) = C : (E^(J) + eps^(J))
      g_i = sum_J c_J sum_j S^(J)_ij G[J, j]     (= div_Y [C : (e_y(X_1:E) + e_Y(U))])
      theta_2 from g by eq. (12) with the mean of g dropped (xi = 0 excluded).
    """
    grad = np.asarray(grad, dtype=np.float64).reshape(6, 3)
    shape = prob.shape
    xg = np.zeros((3, 3) + shape)
    g = np.zeros((3,) + shape)
    for J in range(6):
        u = spectral.displacement_from_strain(correctors[J])           # (3, ...)
        xg += MULT[J] * np.einsum("m...,j->mj...", u, grad[J])
        e_unit = np.zeros(6)
        e_unit[J] = 1.0
        eJ = tensors.tensor_from_engineering(e_unit)
        s = prob.C.contract(correctors[J] + eJ[:, :, None, None, None])
        g += MULT[J] * np.einsum("ij...,j->i...", s, grad[J])
    p2 = prob.C.contract(0.5 * (xg + np.swapaxes(xg, 0, 1)))
    theta = spectral.theta_from_g(g)
    g_mean = g.mean(axis=(1, 2, 3))
    return p2 + theta, p2, theta, g, g_mean


def solve_order1(prob, correctors, grad, scheme="cg", tol=1e-12, max_iter=100000):
    """Strain-gradient problem: returns (eps_2, info) with info['g_mean'],
    info['mean_stress'] = Voigt of <C : eps_2 + p_2>."""
    p_rhs, p2, theta, g, g_mean = order1_rhs(prob, correctors, grad)
    scale = (tensors.l2norm(p2) + tensors.l2norm(g)) / (2.0 * abs(prob.mu0))
    eps, info = _solve(prob, p_rhs, scheme, tol, max_iter, scale)
    info["g_mean"] = g_mean
    info["mean_stress"] = tensors.stress_voigt_from_tensor(
        (prob.C.contract(eps) + p2).mean(axis=(2, 3, 4)))
    return eps, info


def order1_unit_solutions(prob, correctors, scheme="cg", tol=1e-12, max_iter=100000):
    """The 18 order-1 solutions for unit gradient loads G[J, j] = 1 (index
    J * 3 + j): strains eps_2^(J,j) (3,3,...) and their mean stresses."""
    sols, means = [], []
    for J in range(6):
        for j in range(3):
            grad = np.zeros((6, 3))
            grad[J, j] = 1.0
            eps, info = solve_order1(prob, correctors, grad, scheme, tol, max_iter)
            sols.append(eps)
            means.append(info["mean_stress"])
    return sols, np.array(means)


def order2_rhs(prob, correctors, order1_solutions, hess):
    """Right-hand side of the problem of the paper's order alpha = 3 (Sec. 3,
    the definition of p_alpha and g_alpha for alpha >= 3).

    correctors: six order-0 strain fields; order1_solutions: the 18 order-1
    strain fields for unit gradient loads G[J, j] = 1 (index J * 3 + j);
    hess: (6, 3, 3) array H[J, j, m] = d^2 E_kl / dY_j dY_m (symmetric in j, m).
    With u_2 = sum_{J,j} G[J, j] w^(J,j) (w the displacement of the unit
    solution J, j) and G[J, j](Y) = dE_J/dY_j, so that dG[J, j]/dY_m = H[J, j, m]:

      (X_2 . H)_am = sum_{J,j} w^(J,j)_a H[J, j, m]
      p_3 = C : sym(X_2 . H)                                (p_alpha, alpha = 3)
      S_2^(J,j) = C : eps_2^(J,j) + p_2^(J,j),   p_2^(J,j) = C : sym(c_J X_1[:, J] x e_j)
      g_i = sum_{J,j,m} S_2^(J,j)_im H[J, j, m]   (= div_Y [C : (e_y(u_2) + e_Y(u_1))])
      theta_3 from g by eq. (12) with the mean of g dropped.
    Returns (P = p_3 + theta_3, p_3, theta_3, g, <g>).
    """
    hess = np.asarray(hess, dtype=np.float64).reshape(6, 3, 3)
    shape = prob.shape
    v = np.zeros((3, 3) + shape)
    g = np.zeros((3,) + shape)
    x1 = [spectral.displacement_from_strain(correctors[J]) for J in range(6)]
    eye = np.eye(3)
    for J in range(6):
        for j in range(3):
            h = hess[J, j]                                           # (3,) over m
            if not np.any(h):
                continue
            e2 = order1_solutions[J * 3 + j]
            w = spectral.displacement_from_strain(e2)
            v += np.einsum("a...,m->am...", w, h)
            xe = MULT[J] * np.einsum("a...,j->aj...", x1[J], eye[j])   # c_J X_1[:, J] x e_j
            p2 = prob.C.contract(0.5 * (xe + np.swapaxes(xe, 0, 1)))
            s2 = prob.C.contract(e2) + p2
            g += np.einsum("im...,m->i...", s2, h)
    p3 = prob.C.contract(0.5 * (v + np.swapaxes(v, 0, 1)))
    theta = spectral.theta_from_g(g)
    return p3 + theta, p3, theta, g, g.mean(axis=(1, 2, 3))


def solve_order2(prob, correctors, order1_solutions, hess, scheme="cg", tol=1e-12, max_iter=100000):
    """Problem of the paper's order 3: returns (eps_3, info) with info['g_mean']
    and info['mean_stress'] = Voigt of <C : eps_3 + p_3>."""
    p_rhs, p3, theta, g, g_mean = order2_rhs(prob, correctors, order1_solutions, hess)
    scale = (tensors.l2norm(p3) + tensors.l2norm(g)) / (2.0 * abs(prob.mu0))
    eps, info = _solve(prob, p_rhs, scheme, tol, max_iter, scale)
    info["g_mean"] = g_mean
    info["mean_stress"] = tensors.stress_voigt_from_tensor(
        (prob.C.contract(eps) + p3).mean(axis=(2, 3, 4)))
    return eps, info


# ---------------------------------------------------------------------------
# Bounds on the effective stiffness
# ---------------------------------------------------------------------------

def voigt_bound(prob):
    return tensors.voigt66_from_stiffness(prob.C.mean_tensor())


def reuss_bound(prob):
    n = int(np.prod(prob.shape))
    s = np.zeros((6, 6))
    for p, idx in prob.C.index.items():
        s += len(idx) * np.linalg.inv(tensors.voigt66_from_stiffness(prob.C.tensors[p]))
    return np.linalg.inv(s / n)


def hashin_shtrikman_bulk(fractions, k, mu):
    """Hashin-Shtrikman bounds on the bulk modulus for isotropic phases.

    K_HS(mu*) = [ sum_a f_a / (K_a + 4/3 mu*) ]^-1 - 4/3 mu*, with mu* = max mu (upper)
    and min mu (lower)."""
    f = np.asarray(fractions, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)

    def hs(m):
        return 1.0 / np.sum(f / (k + 4.0 * m / 3.0)) - 4.0 * m / 3.0

    return hs(np.min(mu)), hs(np.max(mu))


def bulk_energy_measures(ceff):
    """(I:C_eff:I / 9, 1 / (I:S_eff:I)) from a Voigt 6x6 matrix."""
    ones = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
    kc = ones @ ceff @ ones / 9.0
    ks = 1.0 / (ones @ np.linalg.inv(ceff) @ ones)
    return kc, ks


# ---------------------------------------------------------------------------
# Laminates: exact one-dimensional reductions used as pins
# ---------------------------------------------------------------------------

def laminate_backus(lam, mu, fractions):
    """Effective Voigt stiffness of an isotropic laminate normal to x3 (Backus)."""
    lam = np.asarray(lam, float)
    mu = np.asarray(mu, float)
    f = np.asarray(fractions, float)

    def avg(v):
        return np.sum(f * v)

    c33 = 1.0 / avg(1.0 / (lam + 2 * mu))
    c13 = c33 * avg(lam / (lam + 2 * mu))
    c44 = 1.0 / avg(1.0 / mu)
    c66 = avg(mu)
    c11 = avg(4 * mu * (lam + mu) / (lam + 2 * mu)) + c33 * avg(lam / (lam + 2 * mu)) ** 2
    c12 = c11 - 2 * c66
    c = np.zeros((6, 6))
    c[0, 0] = c[1, 1] = c11
    c[2, 2] = c33
    c[0, 1] = c[1, 0] = c12
    c[0, 2] = c[2, 0] = c[1, 2] = c[2, 1] = c13
    c[3, 3] = c[4, 4] = c44
    c[5, 5] = c66
    return c


def laminate_layers_voigt(c66_layers, fractions):
    """Effective Voigt stiffness (engineering shear) of a laminate of
    anisotropic layers normal to x3, from the layers' 6x6 Voigt matrices.

    Across the layers the traction (sigma_33, sigma_23, sigma_13) and the
    in-plane engineering strains (eps_11, eps_22, gamma_12) are uniform.  With
    the Voigt indices split into N = (33, 23, 13) and T = (11, 22, 12), each
    layer gives e_N = C_NN^-1 (s_N - C_NT e_T) and
    s_T = (C_TT - C_TN C_NN^-1 C_NT) e_T + C_TN C_NN^-1 s_N; averaging e_N
    and s_T over the layers yields
      C*_NN = <C_NN^-1>^-1,          C*_NT = C*_NN <C_NN^-1 C_NT>,
      C*_TT = <C_TT - C_TN C_NN^-1 C_NT> + <C_TN C_NN^-1> C*_NN <C_NN^-1 C_NT>.
    For isotropic layers this reduces to laminate_backus."""
    c = np.asarray(c66_layers, dtype=np.float64).reshape(-1, 6, 6)
    f = np.asarray(fractions, dtype=np.float64)
    N, T = [2, 3, 4], [0, 1, 5]
    cnn = c[:, N][:, :, N]
    cnt = c[:, N][:, :, T]
    ctn = c[:, T][:, :, N]
    ctt = c[:, T][:, :, T]
    inv = np.linalg.inv(cnn)

    def avg(a):
        return np.einsum("l,l...->...", f, a)

    snn = np.linalg.inv(avg(inv))
    a_nt = avg(inv @ cnt)
    a_tn = avg(ctn @ inv)
    out = np.zeros((6, 6))
    out[np.ix_(N, N)] = snn
    out[np.ix_(N, T)] = snn @ a_nt
    out[np.ix_(T, N)] = a_tn @ snn
    out[np.ix_(T, T)] = avg(ctt - ctn @ inv @ cnt) + a_tn @ snn @ a_nt
    return out


def laminate_1d_solve(ctens_profile, pol_profile):
    """Exact discrete solution for a laminate whose data vary along x3 only.

    ctens_profile: (n, 3,3,3,3) stiffness per layer voxel; pol_profile: (n, 3, 3)
    right-hand-side polarization per voxel (constant in x1, x2).
    Equilibrium of (C:eps + P) with eps = sym(e3 x u'(x3)) gives
    Q u' + P[:, 2] = c, Q_ik = C_i3k3, and the periodic zero-mean condition
    <u'> = 0 fixes c = <Q^-1>^-1 <Q^-1 P[:,2]>.  Valid on the discrete grid for
    odd n (no Nyquist mode) - returns eps (n, 3, 3).
    """
    n = ctens_profile.shape[0]
    q = ctens_profile[:, :, 2, :, 2]                  # (n, 3, 3)
    qinv = np.linalg.inv(q)
    pz = pol_profile[:, :, 2]                         # (n, 3)
    c = np.linalg.solve(qinv.mean(axis=0), np.einsum("nik,nk->i", qinv, pz) / n)
    du = np.einsum("nik,nk->ni", qinv, c[None, :] - pz)
    eps = np.zeros((n, 3, 3))
    for i in range(3):
        eps[:, i, 2] += 0.5 * du[:, i]
        eps[:, 2, i] += 0.5 * du[:, i]
    return eps


def antiderivative_1d(g_profile):
    """Zero-mean trigonometric antiderivative along a 1-D periodic grid of
    unit length (odd n): F' = g - <g>.  g_profile (n, ...)."""
    n = g_profile.shape[0]
    gh = fftref.fft(g_profile, axis=0)
    j = np.arange(n)
    k = np.where(j < (n + 1) // 2, j, j - n).astype(float)
    xi = 2 * np.pi * k
    shp = (n,) + (1,) * (g_profile.ndim - 1)
    xi = xi.reshape(shp)
    fh = np.where(xi != 0, gh / (1j * np.where(xi != 0, xi, 1.0)), 0.0)
    return np.real(fftref.ifft(fh, axis=0))
