"""Per-element spectral derivatives, geometry, Q-criterion and |omega| (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Layout: every field is an array ``f[e, k, j, i]`` of shape (E, N+1, N+1, N+1)
with i (the r direction) fastest -- the element-major layout of the Nek data
model that the paper (section 3, DataAdaptor subsection) says NekRS shares
with Nek5000.  Reference coordinates are (r, s, t) along (i, j, k).

Definitions (Deville, Fischer & Mund 2002, ch. 4; Hunt, Wray & Moin 1988):

* reference derivatives, one 1-D contraction with D per direction:
  f_r[e,k,j,i] = sum_m D[i,m] f[e,k,j,m]
  f_s[e,k,j,i] = sum_m D[j,m] f[e,k,m,i]
  f_t[e,k,j,i] = sum_m D[k,m] f[e,m,j,i]
* Jacobian J = d(x,y,z)/d(r,s,t), rows (x_r x_s x_t), (y_..), (z_..);
  det J by cofactor expansion along the first row; J^-1 = adj(J) / det J,
  whose rows are (r_x r_y r_z), (s_x s_y s_z), (t_x t_y t_z);
* physical gradient by the chain rule  df/dx = f_r r_x + f_s s_x + f_t t_x;
* velocity gradient A_ij = d u_i / d x_j, strain S = (A + A^T)/2, rotation
  Omega = (A - A^T)/2, Q = (|Omega|_F^2 - |S|_F^2) / 2,
  omega = (A_32 - A_23, A_13 - A_31, A_21 - A_12), |omega| = sqrt(omega.omega).

Derived quantities are evaluated pointwise inside each element; no averaging
across shared face nodes.
"""

import numpy as np


def ref_derivs(f, d):
    """Return (f_r, f_s, f_t) for ``f`` of shape (E, P, P, P) and D (P, P)."""
    f = np.asarray(f, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    f_r = np.einsum("im,ekjm->ekji", d, f, optimize=True)
    f_s = np.einsum("jm,ekmi->ekji", d, f, optimize=True)
    f_t = np.einsum("km,emji->ekji", d, f, optimize=True)
    return f_r, f_s, f_t


def jacobian(x, y, z, d):
    """Return the 3x3 Jacobian entries as an array of shape (3, 3, E, P, P, P).

    jac[a, b] = d x_a / d r_b with (x_0, x_1, x_2) = (x, y, z) and
    (r_0, r_1, r_2) = (r, s, t).
    """
    rows = [ref_derivs(c, d) for c in (x, y, z)]
    return np.array([[rows[a][b] for b in range(3)] for a in range(3)])


def det3(m):
    """Determinant of stacked 3x3 matrices m[a, b, ...] (first-row cofactors)."""
    return (m[0, 0] * (m[1, 1] * m[2, 2] - m[1, 2] * m[2, 1])
            - m[0, 1] * (m[1, 0] * m[2, 2] - m[1, 2] * m[2, 0])
            + m[0, 2] * (m[1, 0] * m[2, 1] - m[1, 1] * m[2, 0]))


def inverse3(m):
    """Return (adj(m) / det m, det m) for stacked 3x3 matrices m[a, b, ...]."""
    det = det3(m)
    adj = np.empty_like(m)
    # adj[b, a] = cofactor C[a, b]
    adj[0, 0] = m[1, 1] * m[2, 2] - m[1, 2] * m[2, 1]
    adj[0, 1] = -(m[0, 1] * m[2, 2] - m[0, 2] * m[2, 1])
    adj[0, 2] = m[0, 1] * m[1, 2] - m[0, 2] * m[1, 1]
    adj[1, 0] = -(m[1, 0] * m[2, 2] - m[1, 2] * m[2, 0])
    adj[1, 1] = m[0, 0] * m[2, 2] - m[0, 2] * m[2, 0]
    adj[1, 2] = -(m[0, 0] * m[1, 2] - m[0, 2] * m[1, 0])
    adj[2, 0] = m[1, 0] * m[2, 1] - m[1, 1] * m[2, 0]
    adj[2, 1] = -(m[0, 0] * m[2, 1] - m[0, 1] * m[2, 0])
    adj[2, 2] = m[0, 0] * m[1, 1] - m[0, 1] * m[1, 0]
    return adj / det, det


def geometry(x, y, z, d):
    """Return (jinv, det, bad) where jinv[a, b] = d r_a / d x_b.

    ``bad`` is True where det J <= 0 (an inverted or degenerate element),
    which the library reports through its device status word.
    """
    jac = jacobian(x, y, z, d)
    jinv, det = inverse3(jac)
    return jinv, det, ~(det > 0.0)


def physical_gradient(f, jinv, d):
    """Return (df/dx, df/dy, df/dz) by the chain rule."""
    fr, fs, ft = ref_derivs(f, d)
    return tuple(fr * jinv[0, b] + fs * jinv[1, b] + ft * jinv[2, b]
                 for b in range(3))


def derivs(x, y, z, f, d):
    """Physical gradient of one scalar field: (df/dx, df/dy, df/dz), bad."""
    jinv, _, bad = geometry(x, y, z, d)
    return physical_gradient(f, jinv, d), bad


def velocity_gradient(x, y, z, u, v, w, d):
    """Return (A, bad) with A[i, j] = d u_i / d x_j, shape (3, 3, E, P, P, P)."""
    jinv, _, bad = geometry(x, y, z, d)
    rows = [physical_gradient(c, jinv, d) for c in (u, v, w)]
    return np.array([[rows[i][j] for j in range(3)] for i in range(3)]), bad


def q_and_vorticity(a):
    """Hunt's Q = (|Omega|^2 - |S|^2)/2 and |omega| from A[i, j, ...]."""
    at = np.swapaxes(a, 0, 1)
    s = 0.5 * (a + at)
    om = 0.5 * (a - at)
    q = 0.5 * (np.sum(om * om, axis=(0, 1)) - np.sum(s * s, axis=(0, 1)))
    w1 = a[2, 1] - a[1, 2]
    w2 = a[0, 2] - a[2, 0]
    w3 = a[1, 0] - a[0, 1]
    omag = np.sqrt(w1 * w1 + w2 * w2 + w3 * w3)
    return q, omag


def qcrit(x, y, z, u, v, w, d):
    """Full per-point Q-criterion and vorticity magnitude.

    Returns (q, omega_mag, bad) with q, omega_mag shaped like the inputs.
    """
    a, bad = velocity_gradient(x, y, z, u, v, w, d)
    q, omag = q_and_vorticity(a)
    return q, omag, bad


def elem_minmax(f):
    """Per-element (min, max) with NaN treated as -inf, shape (E, 2).

    With this convention an element holds a cell whose corner classes differ
    (some node with f > c and some node without) exactly when max > c and
    not (min > c): a NaN node is never above an isovalue, like -inf.
    """
    f = np.asarray(f)
    g = np.where(np.isnan(f), -np.inf, f).reshape(f.shape[0], -1)
    return np.stack([g.min(axis=1), g.max(axis=1)], axis=1)
