"""Effective tensors of the homogenization hierarchy (Sec. 3) from the GPU
solves: volume averages of the local stresses of the unit problems.

  C  (6 x 6)   order 0: column J = Voigt <C : (E^(J) + eps^(J))> for the unit
               engineering strains e_J (the effective stiffness, eq. (2)).
  B  (6 x 18)  order 1: column J*3 + j = Voigt <C : eps_2 + p_2> for the unit
               gradient load G[J, j] = 1 (dE_J/dY_j, tensor component J); the
               effective third-order (strain-gradient) tensor.  It vanishes for
               centrosymmetric cells.
  D  (6 x 36)  order 2 (optional): column k = Voigt <C : eps_3 + p_3> for the
               unit second gradients H[J, j, m] = H[J, m, j] = 1 over the
               pairs j <= m, in the order of SECOND_PAIRS.
  gB (3 x 18)  <g_2> of each order-1 unit load (= sum over C's columns, a
               consistency check of the order-0 results).

The correctors of each order feed the right-hand sides of the next, as the
hierarchy prescribes; every average is the FP64 reduction the solves already
perform.
"""
import numpy as np

from . import ffth

SECOND_PAIRS = [(J, j, m) for J in range(6) for j in range(3) for m in range(j, 3)]


def second_gradient_unit(k):
    """H (54,) of unit load k of SECOND_PAIRS (symmetric in the derivative indices)."""
    J, j, m = SECOND_PAIRS[k]
    h = np.zeros((6, 3, 3))
    h[J, j, m] = h[J, m, j] = 1.0
    return h.reshape(54)


def effective_tensors(phase, lam0, mu0, lame=None, voigt21=None, order=1, scheme="cg", precision="mixed",
                      tol=1e-8, device="cuda:0", keep_fields=False):
    """Solve the unit problems up to `order` (0, 1 or 2) on one grid; returns a
    dict with C, and B, gB (order >= 1), D (order 2), and the fields if asked."""
    kw = dict(lame=lame, voigt21=voigt21, scheme=scheme, precision=precision, tol=tol, device=device)
    out = {}
    s0 = ffth.Solver(phase, lam0, mu0, nloads=6, **kw)
    eps0, r0 = s0.solve_order0(np.eye(6))
    s0.close()
    out["C"] = np.array([r["mean_stress"] for r in r0]).T
    if order >= 1:
        s1 = ffth.Solver(phase, lam0, mu0, nloads=18, order=1, **kw)
        eps1, r1 = s1.solve_order1(eps0, np.eye(18))
        s1.close()
        out["B"] = np.array([r["mean_stress"] for r in r1]).T
        out["gB"] = np.array([r["g_mean"] for r in r1]).T
    if order >= 2:
        hs = np.stack([second_gradient_unit(k) for k in range(len(SECOND_PAIRS))])
        s2 = ffth.Solver(phase, lam0, mu0, nloads=len(SECOND_PAIRS), order=2, **kw)
        eps2, r2 = s2.solve_order2(eps0, eps1, hs)
        s2.close()
        out["D"] = np.array([r["mean_stress"] for r in r2]).T
        out["gD"] = np.array([r["g_mean"] for r in r2]).T
        if keep_fields:
            out["eps2"] = eps2
    if keep_fields:
        out["eps0"] = eps0
        if order >= 1:
            out["eps1"] = eps1
    return out
