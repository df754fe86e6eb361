"""Spectral finite-element ingredients (paper Sec. III.A, eqn:FEWfns, eqn:cellIntegrals).

Plain, unoptimised float64 code.  Test infrastructure only.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# Legendre polynomials and the two 1-D rules
# ---------------------------------------------------------------------------
def legendre(n: int, x):
    """P_n(x), P_n'(x), P_n''(x) by the three-term recurrence
    (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1} and its derivative forms
    P'_{k+1} = P'_{k-1} + (2k+1) P_k,  P''_{k+1} = P''_{k-1} + (2k+1) P'_k."""
    x = np.asarray(x, dtype=np.float64)
    P = [np.ones_like(x), x.copy()]
    dP = [np.zeros_like(x), np.ones_like(x)]
    ddP = [np.zeros_like(x), np.zeros_like(x)]
    for k in range(1, n):
        P.append(((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1))
        dP.append(dP[k - 1] + (2 * k + 1) * P[k])
        ddP.append(ddP[k - 1] + (2 * k + 1) * dP[k])
    return P[n], dP[n], ddP[n]


def gauss_legendre(nq: int):
    """Gauss-Legendre points (roots of P_nq) and weights 2/((1-x^2) P'_nq(x)^2),
    by Newton iteration from Chebyshev-like starting guesses.  The paper
    integrates cell terms with a tensor GL rule of order n_q (Sec. III.A)."""
    i = np.arange(nq)
    x = np.cos(np.pi * (i + 0.75) / (nq + 0.5))
    for _ in range(100):
        p, dp, _ = legendre(nq, x)
        dx = p / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    _, dp, _ = legendre(nq, x)
    w = 2.0 / ((1.0 - x * x) * dp * dp)
    order = np.argsort(x)
    return x[order], w[order]


def gauss_lobatto(p: int):
    """GLL nodes (+-1 and the roots of P_p') and weights 2/(p(p+1) P_p(x)^2).
    The FE basis is Lagrange on these nodes and the lumped mass M_D is the GLL
    rule at the nodes (Sec. III.A; Sec. III.B.2)."""
    if p == 1:
        return np.array([-1.0, 1.0]), np.array([1.0, 1.0])
    x = -np.cos(np.pi * np.arange(1, p) / p)
    for _ in range(100):
        _, dp, ddp = legendre(p, x)
        dx = dp / ddp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    x = np.concatenate([[-1.0], np.sort(x), [1.0]])
    P, _, _ = legendre(p, x)
    w = 2.0 / (p * (p + 1) * P * P)
    return x, w


def lagrange_tables(nodes, pts):
    """B[i, q] = l_i(t_q) and D[i, q] = l_i'(t_q) for the Lagrange polynomials
    on `nodes`, from the product formula and its derivative (sum over the
    dropped factor)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    pts = np.asarray(pts, dtype=np.float64)
    n = nodes.size
    B = np.ones((n, pts.size))
    D = np.zeros((n, pts.size))
    for i in range(n):
        for j in range(n):
            if j != i:
                B[i] *= (pts - nodes[j]) / (nodes[i] - nodes[j])
        for k in range(n):
            if k == i:
                continue
            term = np.full(pts.size, 1.0 / (nodes[i] - nodes[k]))
            for j in range(n):
                if j != i and j != k:
                    term = term * (pts - nodes[j]) / (nodes[i] - nodes[j])
            D[i] += term
    return B, D


# ---------------------------------------------------------------------------
# Periodic orthorhombic mesh of hexahedral cells
# ---------------------------------------------------------------------------
class Mesh:
    """n_cells[d] cells of size h_d = L_d / n_cells[d] in each direction, with
    degree-p GLL nodes; periodic wrap identifies the faces at 0 and L_d.

    Numbering: global node I = ix + Nx (iy + Ny iz), N_d = n_d p, with
    i_d = (c_d p + a_d) mod N_d for local node i = ax + np (ay + np az) of
    cell e = cx + nx (cy + ny cz).  Spinor dof index 2 I + alpha (eqn:GHEP).
    Quadrature: "gl" is the tensor Gauss-Legendre rule of order n_q
    (eqn:cellIntegrals); "gll" collocates at the GLL nodes (n_q = p + 1).
    """

    def __init__(self, n_cells, box, p, quad="gl", n_q=None):
        self.n_cells = tuple(int(c) for c in n_cells)
        self.box = np.asarray(box, dtype=np.float64)
        self.p = int(p)
        self.np1 = self.p + 1
        self.h = self.box / np.asarray(self.n_cells, dtype=np.float64)
        self.J = float(np.prod(self.h) / 8.0)
        self.N = tuple(c * self.p for c in self.n_cells)
        self.n_nodes = int(np.prod(self.N))
        self.n_cell_total = int(np.prod(self.n_cells))
        self.xi, self.wgll = gauss_lobatto(self.p)
        self.quad = quad
        if quad == "gll":
            self.xq, self.wq1 = self.xi.copy(), self.wgll.copy()
        elif quad == "gl":
            self.xq, self.wq1 = gauss_legendre(int(n_q if n_q else self.p + 1))
        else:
            raise ValueError(quad)
        self.nq = self.xq.size
        self.B1, self.D1 = lagrange_tables(self.xi, self.xq)

        # 3-D tables, local node i = ax + np (ay + np az), point q likewise
        n, m = self.np1, self.nq
        a = np.arange(n)
        ax, ay, az = np.meshgrid(a, a, a, indexing="ij")
        self.loc = np.stack([ax.transpose(2, 1, 0).ravel(), ay.transpose(2, 1, 0).ravel(),
                             az.transpose(2, 1, 0).ravel()], axis=1)        # [n^3][3]
        b = np.arange(m)
        qx, qy, qz = np.meshgrid(b, b, b, indexing="ij")
        self.qloc = np.stack([qx.transpose(2, 1, 0).ravel(), qy.transpose(2, 1, 0).ravel(),
                              qz.transpose(2, 1, 0).ravel()], axis=1)       # [nq^3][3]
        L = self.loc
        Q = self.qloc
        B1, D1 = self.B1, self.D1
        self.Nt = B1[L[:, 0]][:, Q[:, 0]] * B1[L[:, 1]][:, Q[:, 1]] * B1[L[:, 2]][:, Q[:, 2]]
        s = 2.0 / self.h
        self.dNt = [s[0] * D1[L[:, 0]][:, Q[:, 0]] * B1[L[:, 1]][:, Q[:, 1]] * B1[L[:, 2]][:, Q[:, 2]],
                    s[1] * B1[L[:, 0]][:, Q[:, 0]] * D1[L[:, 1]][:, Q[:, 1]] * B1[L[:, 2]][:, Q[:, 2]],
                    s[2] * B1[L[:, 0]][:, Q[:, 0]] * B1[L[:, 1]][:, Q[:, 1]] * D1[L[:, 2]][:, Q[:, 2]]]
        self.wq = (self.wq1[Q[:, 0]] * self.wq1[Q[:, 1]] * self.wq1[Q[:, 2]])  # [nq^3]

    # -- numbering -----------------------------------------------------------
    def cell_coords(self, e):
        nx, ny, _ = self.n_cells
        return e % nx, (e // nx) % ny, e // (nx * ny)

    def cell_nodes(self, e):
        """Global node numbers of the n_p^3 local nodes of cell e (the restriction R^(e))."""
        cx, cy, cz = self.cell_coords(e)
        Nx, Ny, Nz = self.N
        ix = (cx * self.p + self.loc[:, 0]) % Nx
        iy = (cy * self.p + self.loc[:, 1]) % Ny
        iz = (cz * self.p + self.loc[:, 2]) % Nz
        return ix + Nx * (iy + Ny * iz)

    def cell_origin(self, e):
        cx, cy, cz = self.cell_coords(e)
        return np.array([cx, cy, cz], dtype=np.float64) * self.h

    def quad_points(self, e):
        """Physical quadrature points r_q^(e) = origin + (xi_q + 1) h / 2, [nq^3][3]."""
        o = self.cell_origin(e)
        Q = self.qloc
        return np.stack([o[d] + (self.xq[Q[:, d]] + 1.0) * self.h[d] / 2.0 for d in range(3)], axis=1)

    def all_quad_points(self):
        return np.stack([self.quad_points(e) for e in range(self.n_cell_total)])

    def node_coords(self):
        """Physical coordinates of all global nodes, [M][3]."""
        out = []
        for d in range(3):
            i = np.arange(self.N[d])
            c, a = i // self.p, i % self.p
            out.append(c * self.h[d] + (self.xi[a] + 1.0) * self.h[d] / 2.0)
        X, Y, Z = np.meshgrid(out[0], out[1], out[2], indexing="ij")
        return np.stack([X.transpose(2, 1, 0).ravel(), Y.transpose(2, 1, 0).ravel(),
                         Z.transpose(2, 1, 0).ravel()], axis=1)

    def lumped_mass(self):
        """M_D: GLL quadrature at the nodes makes the overlap diagonal,
        M_I = sum over cells containing I of w_ax w_ay w_az J (Sec. III.B.2)."""
        wl = self.wgll[self.loc[:, 0]] * self.wgll[self.loc[:, 1]] * self.wgll[self.loc[:, 2]] * self.J
        M = np.zeros(self.n_nodes)
        for e in range(self.n_cell_total):
            np.add.at(M, self.cell_nodes(e), wl)
        return M
