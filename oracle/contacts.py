"""Contact (collision) projection of the local step (FP64).

Test infrastructure only (see the package docstring).

Colliding neighbours are handed to the solid solver from outside (the fluid
side exchanges them, Implementation and architecture; their strength is the
material's collision weight, section "RBC collision at an obstacle"). Reading:
the neighbourhood of a cell is a list of contact points y_j on the other
surfaces (neighbouring cells or obstacles), each with the unit outward normal
n_j of that surface, in the cell's coordinates. Every vertex carries one
contact potential (w_c/2) dist^2(q_v, C_v), where C_v is the half-space
{p : (p - y_k) . n_k >= 0} of the contact point y_k nearest to q_v (smallest
index on ties): the closest point of C_v is q_v itself when the vertex is
outside, else its projection onto the tangent plane. Because every vertex
carries the potential (inactive ones project onto themselves), its selection
matrix is the identity and the system matrix only gains w_c I: the global
step keeps its constant matrix.
"""
from __future__ import annotations

import numpy as np


def nearest_contact(q: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Index of the contact point nearest to each vertex (ties: smallest index)."""
    d2 = np.sum((q[:, None, :] - pts[None, :, :]) ** 2, axis=2)  # [N, K]
    return np.argmin(d2, axis=1)  # first minimum on ties


def project_contacts(q: np.ndarray, pts: np.ndarray, nrm: np.ndarray) -> np.ndarray:
    """Closest point of each vertex in its contact half-space ([N, 3])."""
    if pts.shape[0] == 0:
        return q.copy()
    k = nearest_contact(q, pts)
    y, n = pts[k], nrm[k]
    s = np.sum((q - y) * n, axis=1)  # signed distance to the tangent plane
    return q - np.minimum(s, 0.0)[:, None] * n
