"""Self-consistent initial fields of an externally injected relativistic
electron bunch, plain FP64 numpy/scipy (the oracle).

TEST INFRASTRUCTURE ONLY: imported by the test suite; it imports nothing
from the GPU package.

What is computed (Sec. 3, last paragraph of the numerical implementation:
the field initialisation for external injection carries over to cylindrical
symmetry; the paper points to the relativistic Poisson method of its
references and gives no equation).  Reading R27, written out here:

  * the bunch moves along x with velocity beta (gamma = 1/sqrt(1 - beta^2));
    its fields are those of the charge at rest in its own frame, boosted:
        (1/gamma^2) d2phi/dx2 + (1/r) d/dr (r dphi/dr) = -rho,
        E_x = -(1/gamma^2) dphi/dx,  E_r = -dphi/dr,  B_theta = beta E_r
    (mode 0 only: an axisymmetric bunch);
  * discretised on the Yee grid so that the discrete Gauss law of the PIC
    loop holds exactly: phi on the primal nodes (i, j), zero on the x ends
    and at r_max (the boundaries of the field solver),
        E_x(i+1/2, j) = -(phi(i+1, j) - phi(i, j)) / (gamma^2 dx),
        E_r(i, j+1/2) = -(phi(i, j+1) - phi(i, j)) / dr,
    and div E = rho at every interior node with the divergence of the field
    update (axial differences over dx; radial face areas A(j+1/2) =
    2 pi (j+1/2) dr dx over the node volume V_j, V_0 = pi dr^2 dx / 4);
  * rho V_j is the bunch's charge deposited with the loop's particle shape
    (sum q w S, q = -1; linear or quadratic, the latter folded across the
    axis); nodes on the boundaries (i = 0, nx or j = nr) hold no unknown;
  * B_theta at (i+1/2, j+1/2) is beta times the mean of E_r at i and i+1
    (the magnetic field of the moving charge at the same instant); the
    time-averaged B-bar is the same field.

The linear system (multiplied by V_j) is symmetric positive definite and is
solved directly (scipy.sparse.linalg.spsolve).  Pinned by
tests/test_oracle_bunch.py: the discrete Gauss law against the test's own
deposit, the radial field of a long uniform cylinder (E_r = rho r / 2
inside, Q' / (2 pi r) outside), the 1/gamma^2 scaling of E_x, the total
charge, and the cancellation of the radial self-force on a co-moving
electron to 1/gamma^2 through one momentum step of the oracle's pusher.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

Q_ELECTRON = -1.0


def _weights(u, order):
    """(first node, weights) of the shape of order 1 or 2 at node coordinate u."""
    if order == 2:
        m = np.floor(u + 0.5)
        d = u - m
        return m.astype(np.int64) - 1, [0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2]
    f = np.floor(u)
    return f.astype(np.int64), [1.0 - (u - f), u - f]


def charge_nodes(cfg, parts, shift=0):
    """q sum w S on the primal nodes, (nx+1) x (nr+1); contributions below the
    axis fold onto their mirror rows (primal row -j mirrors row j)."""
    nx, nr, dx, dr = cfg["nx"], cfg["nr"], cfg["dx"], cfg["dr"]
    order = 2 if cfg.get("shape_order", 1) == 2 else 1
    ux = np.asarray(parts["x"], float) / dx - shift
    ur = np.hypot(parts["y"], parts["z"]) / dr
    ix, wx = _weights(ux, order)
    jr, wr = _weights(ur, order)
    out = np.zeros((nx + 1, nr + 1))
    w = np.asarray(parts["w"], float)
    for a, wa in enumerate(wx):
        for b, wb in enumerate(wr):
            i = ix + a
            j = jr + b
            j = np.where(j < 0, -j, j)
            ok = (i >= 0) & (i <= nx) & (j >= 0) & (j <= nr)
            np.add.at(out, (i[ok], j[ok]), Q_ELECTRON * w[ok] * wa[ok] * wb[ok])
    return out


def volumes(cfg):
    dx, dr, nr = cfg["dx"], cfg["dr"], cfg["nr"]
    j = np.arange(nr + 1)
    V = 2 * np.pi * j * dr * dr * dx
    V[0] = np.pi * dr * dr * dx / 4
    A = 2 * np.pi * (j + 0.5) * dr * dx  # radial face at r_{j+1/2}
    return V, A


def bunch_fields(cfg, parts, beta, shift=0):
    """(E_x, E_r, B_theta, phi, rho V) of the bunch on the window-relative
    grids of the loop: E_x at (i+1/2, j), E_r at (i, j+1/2), B_theta at
    (i+1/2, j+1/2), each (nx+1) x (nr+1) with the unused last column or row
    zero."""
    nx, nr, dx, dr = cfg["nx"], cfg["nr"], cfg["dx"], cfg["dr"]
    g2 = 1.0 - beta * beta
    V, A = volumes(cfg)
    qv = charge_nodes(cfg, parts, shift)
    ni, nj = nx - 1, nr  # unknowns: i = 1..nx-1, j = 0..nr-1
    idx = lambda i, j: (i - 1) * nj + j
    rows, cols, vals = [], [], []
    rhs = np.zeros(ni * nj)
    for i in range(1, nx):
        for j in range(nr):
            k = idx(i, j)
            cx = V[j] * g2 / (dx * dx)  # (1/gamma^2) V_j / dx^2
            diag = 2.0 * cx
            for i2 in (i - 1, i + 1):
                if 1 <= i2 <= nx - 1:
                    rows.append(k), cols.append(idx(i2, j)), vals.append(-cx)
            up = A[j] / dr
            diag += up
            if j + 1 <= nr - 1:
                rows.append(k), cols.append(idx(i, j + 1)), vals.append(-up)
            if j >= 1:
                dn = A[j - 1] / dr
                diag += dn
                rows.append(k), cols.append(idx(i, j - 1)), vals.append(-dn)
            rows.append(k), cols.append(k), vals.append(diag)
            rhs[k] = qv[i, j]
    K = sp.csr_matrix((vals, (rows, cols)), shape=(ni * nj, ni * nj))
    sol = spla.spsolve(K.tocsc(), rhs)
    phi = np.zeros((nx + 1, nr + 1))
    phi[1:nx, 0:nr] = sol.reshape(ni, nj)
    ex = np.zeros((nx + 1, nr + 1))
    er = np.zeros((nx + 1, nr + 1))
    bt = np.zeros((nx + 1, nr + 1))
    ex[:nx, :] = -(phi[1:, :] - phi[:-1, :]) * g2 / dx
    er[:, :nr] = -(phi[:, 1:] - phi[:, :-1]) / dr
    bt[:nx, :nr] = beta * 0.5 * (er[:nx, :nr] + er[1:, :nr])
    return ex, er, bt, phi, qv
