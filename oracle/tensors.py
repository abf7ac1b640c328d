"""Tensor algebra for the oracle (test infrastructure only).

Fields are full 3x3 tensors of shape (3, 3, n0, n1, n2); the grid axis d
carries the coordinate x_{d+1}.  Stiffnesses are full 4th-order tensors
C_ijkl of shape (3, 3, 3, 3).

Voigt input/output convention: a 6-vector lists (11, 22, 33, 23, 13, 12).
Strain-like *fields* keep tensor components in that order; the macroscopic
strain E and stiffness tables use engineering shear (gamma = 2 eps), so a
6x6 Voigt stiffness maps an engineering strain vector to the stress vector.
"""
import numpy as np

VOIGT_PAIRS = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def isotropic_stiffness(lam, mu):
    """C_ijkl = lam d_ij d_kl + mu (d_ik d_jl + d_il d_jk)  (reference medium, Sec. 2)."""
    d = np.eye(3)
    return (lam * np.einsum("ij,kl->ijkl", d, d)
            + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def voigt_index(i, j):
    for a, (p, q) in enumerate(VOIGT_PAIRS):
        if (i, j) in ((p, q), (q, p)):
            return a
    raise ValueError


def stiffness_from_voigt66(c66):
    """Full tensor from a symmetric 6x6 Voigt matrix (engineering shear)."""
    c = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for m in range(3):
                    c[i, j, k, m] = c66[voigt_index(i, j), voigt_index(k, m)]
    return c


def voigt66_from_stiffness(c):
    out = np.zeros((6, 6))
    for a, (i, j) in enumerate(VOIGT_PAIRS):
        for b, (k, m) in enumerate(VOIGT_PAIRS):
            out[a, b] = c[i, j, k, m]
    return out


def voigt66_from_upper21(v21):
    """21 upper-triangular Voigt coefficients, row-major: C11 C12 .. C16 C22 .. C66."""
    m = np.zeros((6, 6))
    idx = 0
    for a in range(6):
        for b in range(a, 6):
            m[a, b] = m[b, a] = v21[idx]
            idx += 1
    return m


def tensor_from_engineering(e6):
    """Macroscopic strain tensor from an engineering Voigt 6-vector."""
    e6 = np.asarray(e6, dtype=np.float64)
    t = np.zeros((3, 3))
    for a, (i, j) in enumerate(VOIGT_PAIRS):
        v = e6[a] if a < 3 else 0.5 * e6[a]
        t[i, j] = t[j, i] = v
    return t


def field_from_voigt6(f6):
    """(6, ...) tensor-component field -> (3, 3, ...) symmetric field."""
    f6 = np.asarray(f6, dtype=np.float64)
    out = np.zeros((3, 3) + f6.shape[1:])
    for a, (i, j) in enumerate(VOIGT_PAIRS):
        out[i, j] = f6[a]
        out[j, i] = f6[a]
    return out


def voigt6_from_field(f):
    """(3, 3, ...) field -> (6, ...) tensor components (11, 22, 33, 23, 13, 12)."""
    return np.stack([f[i, j] for (i, j) in VOIGT_PAIRS])


def stress_voigt_from_tensor(s):
    return np.array([s[i, j] for (i, j) in VOIGT_PAIRS])


class StiffnessField:
    """C(x) = table[phase(x)] for a phase-id voxel array (the stiffness field of Sec. 2)."""

    def __init__(self, phase, tensors):
        self.phase = np.asarray(phase)
        self.tensors = np.asarray(tensors, dtype=np.float64)   # (nphases, 3, 3, 3, 3)
        self.shape = self.phase.shape
        ids = self.phase.ravel()
        self.index = {}
        for p in np.unique(ids):
            self.index[int(p)] = np.nonzero(ids == p)[0]

    @classmethod
    def from_lame(cls, phase, lame):
        lame = np.asarray(lame, dtype=np.float64).reshape(-1, 2)
        return cls(phase, np.stack([isotropic_stiffness(l, m) for l, m in lame]))

    @classmethod
    def from_voigt21(cls, phase, v21):
        v21 = np.asarray(v21, dtype=np.float64).reshape(-1, 21)
        return cls(phase, np.stack([stiffness_from_voigt66(voigt66_from_upper21(r)) for r in v21]))

    def contract(self, eps, minus=None):
        """sigma_ij(x) = (C(x) - minus)_ijkl eps_kl(x)  (Hooke's law, eq. (2))."""
        flat = eps.reshape(3, 3, -1)
        out = np.zeros_like(flat)
        for p, idx in self.index.items():
            c = self.tensors[p] if minus is None else self.tensors[p] - minus
            out[:, :, idx] = np.einsum("ijkl,klm->ijm", c, flat[:, :, idx])
        return out.reshape(eps.shape)

    def contract_const(self, e, minus=None):
        """C(x):E for a constant tensor E."""
        n = int(np.prod(self.shape))
        out = np.zeros((3, 3, n))
        for p, idx in self.index.items():
            c = self.tensors[p] if minus is None else self.tensors[p] - minus
            out[:, :, idx] = np.einsum("ijkl,kl->ij", c, e)[:, :, None]
        return out.reshape((3, 3) + self.shape)

    def mean_tensor(self):
        """Volume average <C> (Voigt bound)."""
        n = int(np.prod(self.shape))
        return sum(len(idx) * self.tensors[p] for p, idx in self.index.items()) / n


def frobenius(a, b):
    """Full contraction a:b summed over the grid (off-diagonals counted twice)."""
    return float(np.sum(a * b))


def l2norm(a):
    return float(np.sqrt(np.sum(a * a)))
