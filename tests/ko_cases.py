"""Test inputs for the Kelvin-Onsager enforcement (Eqs. 32-35), built from
the oracle alone (shared by the oracle pins and the GPU parity tests)."""
import numpy as np

import oracle


def planted_ko_case(prob, T, c, seed=5):
    """Random I, J, F and a G for which alpha_ph / T is c times the drag part
    of sigma S, so that Eq. 35 holds exactly at lambda = c.  G is found from
    the linearity of alpha_ph in G: the oracle's own tensors of the nine
    responses G = E_bb' v_ph span the map, which is then solved for G."""
    rng = np.random.default_rng(seed)
    M = prob.nstates
    I = rng.standard_normal((M, 3)) * 1e-8
    J = rng.standard_normal((M, 3)) * 1e-8
    F = rng.standard_normal(prob.v_ph.shape) * 1e-8
    zero = np.zeros_like(F)
    I_drag = I - ((prob.eps - prob.mu) / T)[:, None] * J
    target = c * T * oracle.transport_tensors(prob, T, I_drag, J, F, zero)["sigmaS"]
    A = np.zeros((9, 9))
    for k in range(9):
        E = np.zeros((3, 3))
        E.flat[k] = 1.0
        A[:, k] = oracle.transport_tensors(prob, T, I, J, F, prob.v_ph @ E.T)["alpha_ph"].ravel()
    m = np.linalg.solve(A, target.ravel())
    return I, J, F, prob.v_ph @ m.reshape(3, 3).T
