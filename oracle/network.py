"""DC network algebra of the contingency model (Section II-E, "Contingency
evaluation").

Definitions followed here
-------------------------
* A branch carries DC flow f_l = y_l (theta_from - theta_to) with
  y_l = -b_l^sr = x_l / (r_l^2 + x_l^2), the series susceptance in the flow
  formula of Section II-E (the text also calls Y_x "inverse line reactances";
  the flow formula is taken as the definition).
* E is the signed branch-bus incidence matrix (+1 at the from bus, -1 at the
  to bus), so nodal injections are E^T f and Y_b = E^T diag(y) E.
* Deleting the reference bus gives the reduced system of eq. (Yb_solve):
  theta_hat = Yhat_b^{-1} p_hat, flows p = diag(y) Ehat theta_hat (eq. p_flow).
* Injections are balanced by a uniform slack before the solve, p_bar =
  p_inj - mean(p_inj), the slack rule whose gradient eq. (correction) states.
  With balanced injections the flows do not depend on the reference bus.
* Contingency k removes one branch; its flows are the same solve on the
  network without that branch.  The rank-1 form (eq. rank_correct) is the
  Sherman-Morrison form of that re-solve; expressed on flows it becomes the
  line outage distribution factors computed by ``lodf``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

__all__ = ["incidence", "susceptance", "is_connected", "bridges_bruteforce",
           "dc_flows_solve", "isf_matrix", "lodf_matrix", "outage_flows"]


def incidence(n_bus, br_from, br_to):
    """Dense signed incidence E [L, N]: +1 at the from bus, -1 at the to bus."""
    L = len(br_from)
    E = np.zeros((L, n_bus))
    E[np.arange(L), br_from] = 1.0
    E[np.arange(L), br_to] = -1.0
    return E


def susceptance(br_r, br_x):
    """y_l = -b^sr_l = x / (r^2 + x^2)."""
    return br_x / (br_r * br_r + br_x * br_x)


def is_connected(n_bus, br_from, br_to, mask=None):
    if mask is None:
        mask = np.ones(len(br_from), dtype=bool)
    a = np.asarray(br_from)[mask]
    b = np.asarray(br_to)[mask]
    g = sp.coo_matrix((np.ones(a.shape[0]), (a, b)), shape=(n_bus, n_bus))
    ncomp, _ = connected_components(g, directed=False)
    return ncomp == 1


def bridges_bruteforce(n_bus, br_from, br_to):
    """Boolean [L]: True where removing the branch disconnects the grid.

    Brute force by definition: drop each branch and test connectivity.
    """
    L = len(br_from)
    out = np.zeros(L, dtype=bool)
    for l in range(L):
        m = np.ones(L, dtype=bool)
        m[l] = False
        out[l] = not is_connected(n_bus, br_from, br_to, m)
    return out


def dc_flows_solve(E, y, p_bar, ref=0):
    """Flows for injections p_bar [..., N] by the reduced solve.

    theta_hat = Yhat^{-1} p_hat (eq. Yb_solve); f = diag(y) Ehat theta_hat
    (eq. p_flow).  p_bar must sum to zero over buses for the result to be a
    flow that meets every injection (Kirchhoff: E^T f = p_bar).
    """
    keep = np.ones(E.shape[1], dtype=bool)
    keep[ref] = False
    Eh = E[:, keep]
    Yh = Eh.T @ (y[:, None] * Eh)
    p = np.atleast_2d(p_bar)[:, keep]
    th = np.linalg.solve(Yh, p.T).T
    f = (th @ Eh.T) * y[None, :]
    return f.reshape(np.shape(p_bar)[:-1] + (E.shape[0],))


def isf_matrix(E, y, ref=0):
    """Injection shift factors [L, N]: f = ISF @ p_bar; ref column is zero.

    ISF = diag(y) Ehat Yhat^{-1}, the linear map of eqs. (Yb_solve)-(p_flow).
    """
    keep = np.ones(E.shape[1], dtype=bool)
    keep[ref] = False
    Eh = E[:, keep]
    Yh = Eh.T @ (y[:, None] * Eh)
    # ISF_hat^T = Yhat^{-1} Ehat^T diag(y)   (Yhat symmetric)
    isf_h = np.linalg.solve(Yh, (Eh * y[:, None]).T).T
    isf = np.zeros(E.shape)
    isf[:, keep] = isf_h
    return isf


def lodf_matrix(isf, br_from, br_to, ctg):
    """Line outage distribution factors [L, K] for outaged branches ctg.

    PTDF_{l,k} = ISF[l, from(k)] - ISF[l, to(k)] is the flow on l per unit
    transferred from the from bus to the to bus of k.  After k opens, its
    pre-outage flow F_k is re-routed: F_l' = F_l + LODF_{l,k} F_k with
    LODF_{l,k} = PTDF_{l,k} / (1 - PTDF_{k,k}) and LODF_{k,k} = -1.  This is
    eq. (rank_correct) mapped from angles to flows.
    """
    ctg = np.asarray(ctg)
    ptdf = isf[:, br_from[ctg]] - isf[:, br_to[ctg]]        # [L, K]
    denom = 1.0 - ptdf[ctg, np.arange(ctg.shape[0])]
    lodf = ptdf / denom[None, :]
    lodf[ctg, np.arange(ctg.shape[0])] = -1.0
    return lodf


def outage_flows(E, y, p_bar, k, ref=0):
    """Post-outage flows [..., L] with branch k removed (flow on k is 0).

    The plain definition of a contingency flow: re-solve the network that
    lacks branch k.
    """
    L = E.shape[0]
    m = np.ones(L, dtype=bool)
    m[k] = False
    f_k = dc_flows_solve(E[m], y[m], p_bar, ref)
    out = np.zeros(np.shape(p_bar)[:-1] + (L,))
    out[..., m] = f_k
    return out
