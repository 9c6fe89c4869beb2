"""The SIPG Laplacian of Section 2: explicit assembly and a naive matrix-free product.

Test infrastructure (see oracle/__init__.py).

Weak form (Section 2, eq. discrete_laplace), per element K and test function
phi_i, with n the outward unit normal of K on face F, {{v}} = (v- + v+)/2 and
[[v]] = n (v- - v+):
    (grad phi_i, grad u)_K
  + sum_F  < phi_i n, sigma [[u]] >_F - < phi_i n, {{grad u}} >_F
         - < grad phi_i / 2, [[u]] >_F .
Homogeneous Dirichlet boundaries use the mirror principle u+ = -u-; the
gradient is mirrored as grad u+ = grad u- (reading: the paper states only the
value; this choice keeps the form symmetric and consistent).

Penalty (Section 2 gives sigma = (p+1)^2 / h): sigma_F = eta (k+1)^2 / h_F with
1/h_F = max(|F| / |K-|, |F| / |K+|) (|K-| alone on boundary faces), all
measures by the same quadrature; on a Cartesian cell of size h this is
eta (k+1)^2 / h.

All integrals use the tensor Gauss formula with k+1 points per direction
(Section 3).  The tensor-product basis is phi_i(xi) = prod_t phi_{i_t}(xi_t)
(eq. phi_tensor) with the in-cell index i = i1 + n i2 + n^2 i3, n = k+1, and
the global vector is stored cell by cell: dof = cell * n^3 + i.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import basis as b1d
from .mesh import map_points, cell_coords


def tensor_eval(basis: b1d.Basis1D, pts: np.ndarray):
    """Values [Q, n^3] and reference gradients [3, Q, n^3] of all tensor-product
    shape functions at reference points pts [Q, 3] (eq. phi_tensor)."""
    n = basis.degree + 1
    V = [basis.values(pts[:, t]) for t in range(3)]    # [Q, n] each
    D = [basis.derivs(pts[:, t]) for t in range(3)]
    Q = pts.shape[0]

    def comb(a, b_, c):
        # out[q, i3, i2, i1] = a[q, i1] b[q, i2] c[q, i3]
        return np.einsum("qa,qb,qc->qcba", a, b_, c).reshape(Q, n ** 3)

    val = comb(V[0], V[1], V[2])
    grad = np.stack([comb(D[0], V[1], V[2]),
                     comb(V[0], D[1], V[2]),
                     comb(V[0], V[1], D[2])])
    return val, grad


def _tangential(d):
    return [t for t in range(3) if t != d]


class SIPG:
    """Discrete SIPG operator on a `workloads.Mesh` with degree k, penalty
    factor eta and a 1D basis ("hermite_like" or "nodal_gl").

    `cells` restricts the rows to a subset of cells (the metric terms are
    then evaluated for those cells only); apply_naive then takes the full
    vector and returns the rows of those cells."""

    def __init__(self, mesh, k: int, eta: float = 2.0, basis: str = "hermite_like", cells=None):
        self.mesh = mesh
        self.all_cells = cells is None
        self.cells = np.arange(mesh.ncells) if cells is None else np.asarray(cells, dtype=np.int64)
        self.k = int(k)
        self.n = self.k + 1
        self.eta = float(eta)
        self.basis = b1d.make_basis(basis, self.k)
        self.nq = self.k + 1
        self.ncells = len(self.cells)
        self.ndofs = self.ncells * self.n ** 3
        self.ncells_total = mesh.ncells
        xq, wq = b1d.gauss(self.nq)
        self.xq, self.wq = xq, wq
        nq = self.nq
        # cell quadrature points, q = q1 + nq q2 + nq^2 q3
        g3, g2, g1 = np.meshgrid(xq, xq, xq, indexing="ij")
        self.cell_pts = np.stack([g1.ravel(), g2.ravel(), g3.ravel()], axis=1)
        w3, w2, w1 = np.meshgrid(wq, wq, wq, indexing="ij")
        self.cell_w = (w1 * w2 * w3).ravel()
        self.cell_val, self.cell_grad = tensor_eval(self.basis, self.cell_pts)
        # face quadrature points: face (d, s) lies at xi_d = s; tangential
        # directions t1 < t2, point index qt1 + nq qt2.
        self.face_pts = {}
        self.face_eval = {}
        ta, tb = np.meshgrid(xq, xq, indexing="xy")  # ta varies fastest
        wa, wb = np.meshgrid(wq, wq, indexing="xy")
        self.face_w = (wa * wb).ravel()
        for d in range(3):
            t1, t2 = _tangential(d)
            for s in (0, 1):
                pts = np.zeros((nq * nq, 3))
                pts[:, d] = float(s)
                pts[:, t1] = ta.ravel()
                pts[:, t2] = tb.ravel()
                self.face_pts[(d, s)] = pts
                self.face_eval[(d, s)] = tensor_eval(self.basis, pts)
        self._geometry()

    # ------------------------------------------------------------------
    def neighbor(self, d: int, s: int) -> np.ndarray:
        """Cell across face (d, s) of every row cell, -1 on the domain boundary."""
        c = self.cells
        idx = list(cell_coords(self.mesh, c))
        step = 1 if s == 1 else -1
        j = idx[d] + step
        ok = (j >= 0) & (j < self.mesh.n[d])
        idx[d] = np.where(ok, j, 0)
        nb = idx[0] + self.mesh.n[0] * (idx[1] + self.mesh.n[1] * idx[2])
        return np.where(ok, nb, -1)

    def volumes(self, cells) -> np.ndarray:
        """|K| = sum_q det J w_q for the given cells."""
        _, J = map_points(self.mesh, np.asarray(cells), self.cell_pts)
        return np.sum(np.linalg.det(J) * self.cell_w, axis=1)

    def _geometry(self):
        cells = self.cells
        _, J = map_points(self.mesh, cells, self.cell_pts)        # [C, Q, 3, 3]
        detJ = np.linalg.det(J)
        if np.any(detJ <= 0):
            raise ValueError("mesh map is not orientation preserving")
        Jinv = np.linalg.inv(J)
        # merged metric J^-1 J^-T det(J) w_q (eq. integral_laplace)
        self.cell_G = (Jinv @ np.swapaxes(Jinv, -1, -2)) * (detJ * self.cell_w)[..., None, None]
        self.cell_volume = np.sum(detJ * self.cell_w, axis=1)
        self.faces = {}
        for d in range(3):
            for s in (0, 1):
                pts = self.face_pts[(d, s)]
                _, Jf = map_points(self.mesh, cells, pts)         # own side
                Jfi = np.linalg.inv(Jf)
                JinvT = np.swapaxes(Jfi, -1, -2)
                ed = np.zeros(3)
                ed[d] = 1.0
                m = JinvT @ ed                                     # J^-T e_d  [C, Qf, 3]
                mn = np.linalg.norm(m, axis=-1)
                sign = 1.0 if s == 1 else -1.0
                normal = sign * m / mn[..., None]
                JxW = np.linalg.det(Jf) * mn * self.face_w         # Nanson's formula
                area = JxW.sum(axis=1)
                nb = self.neighbor(d, s)
                # neighbour Jacobian at the same points, seen from its side 1-s
                pts_nb = self.face_pts[(d, 1 - s)]
                _, Jnb = map_points(self.mesh, np.where(nb >= 0, nb, 0), pts_nb)
                JnbinvT = np.swapaxes(np.linalg.inv(Jnb), -1, -2)
                inv_h = area / self.cell_volume
                vol_nb = self.volumes(np.where(nb >= 0, nb, 0))
                inv_h_nb = np.where(nb >= 0, area / vol_nb, 0.0)
                sigma = self.eta * (self.k + 1) ** 2 * np.maximum(inv_h, inv_h_nb)
                self.faces[(d, s)] = dict(JxW=JxW, normal=normal, JinvT=JinvT,
                                          JinvT_nb=JnbinvT, nb=nb, sigma=sigma)

    # ------------------------------------------------------------------
    def local_blocks(self):
        """Dense blocks (row cell, column cell, n^3 x n^3 block) of A."""
        C, n3 = self.ncells, self.n ** 3
        Gr = self.cell_grad                                       # [3, Q, n3]
        # cell term: sum_ab Gr_a^T diag(G_ab) Gr_b
        Akk = np.zeros((C, n3, n3))
        for a in range(3):
            for b_ in range(3):
                Akk += np.matmul(Gr[a].T[None], self.cell_G[:, :, a, b_, None] * Gr[b_][None])
        offdiag = []
        for (d, s), f in self.faces.items():
            val, grad = self.face_eval[(d, s)]                    # own side
            val_nb, grad_nb = self.face_eval[(d, 1 - s)]          # neighbour side
            JxW, nrm, sig = f["JxW"], f["normal"], f["sigma"]
            # n . grad phi = (J^-T grad_xi phi) . n
            ng = np.einsum("cqab,bqi,cqa->cqi", f["JinvT"], grad, nrm)    # [C,Qf,n3]
            ng_nb = np.einsum("cqab,bqi,cqa->cqi", f["JinvT_nb"], grad_nb, nrm)
            interior = f["nb"] >= 0
            w = JxW
            V = np.broadcast_to(val, ng.shape)
            Vn = np.broadcast_to(val_nb, ng.shape)
            # boundary faces: mirror principle doubles penalty and consistency terms
            fac = np.where(interior, 1.0, 2.0)
            Akk += np.einsum("cq,cqi,cqj->cij", w * (fac * sig)[:, None], V, V)
            Akk -= 0.5 * fac[:, None, None] * (np.einsum("cq,cqi,cqj->cij", w, V, ng)
                                               + np.einsum("cq,cqi,cqj->cij", w, ng, V))
            ci = np.nonzero(interior)[0]
            if len(ci):
                wi = w[ci]
                blk = (-np.einsum("cq,cqi,cqj->cij", wi * sig[ci][:, None], V[ci], Vn[ci])
                       - 0.5 * np.einsum("cq,cqi,cqj->cij", wi, V[ci], ng_nb[ci])
                       + 0.5 * np.einsum("cq,cqi,cqj->cij", wi, ng[ci], Vn[ci]))
                offdiag.append((ci, f["nb"][ci], blk))
        return Akk, offdiag

    def assemble(self) -> sp.csr_matrix:
        """A_ij = a_h(phi_j, phi_i) as a CSR matrix, float64."""
        if not self.all_cells:
            raise ValueError("assemble() needs the operator on all cells")
        C, n3 = self.ncells, self.n ** 3
        Akk, offdiag = self.local_blocks()
        rows = [np.arange(C)]
        cols = [np.arange(C)]
        data = [Akk]
        for ci, cj, blk in offdiag:
            rows.append(ci)
            cols.append(cj)
            data.append(blk)
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
        data = np.concatenate(data)
        A = sp.coo_matrix((C, C))
        # expand blocks to scalar coordinates
        ii, jj = np.meshgrid(np.arange(n3), np.arange(n3), indexing="ij")
        R = (rows[:, None, None] * n3 + ii[None]).ravel()
        Cc = (cols[:, None, None] * n3 + jj[None]).ravel()
        A = sp.coo_matrix((data.ravel(), (R, Cc)), shape=(C * n3, C * n3)).tocsr()
        A.sum_duplicates()
        return A

    # ------------------------------------------------------------------
    def apply_naive(self, x: np.ndarray) -> np.ndarray:
        """y = A x evaluated matrix-free at the quadrature points, with dense
        per-cell evaluation matrices (no sum factorization)."""
        C, n3 = self.ncells, self.n ** 3
        Uall = np.asarray(x, dtype=np.float64).reshape(self.ncells_total, n3)
        U = Uall if self.all_cells else Uall[self.cells]
        Gr = self.cell_grad
        gu = np.stack([U @ Gr[a].T for a in range(3)], axis=-1)          # [C, Q, 3]
        t = np.einsum("cqab,cqb->cqa", self.cell_G, gu)
        Y = sum(t[..., a] @ Gr[a] for a in range(3))
        for (d, s), f in self.faces.items():
            val, grad = self.face_eval[(d, s)]
            val_nb, grad_nb = self.face_eval[(d, 1 - s)]
            nb = f["nb"]
            interior = nb >= 0
            Unb = Uall[np.where(interior, nb, 0)]
            um = U @ val.T                                                 # [C, Qf]
            gm = np.einsum("cqab,cqb->cqa", f["JinvT"],
                           np.stack([U @ grad[a].T for a in range(3)], axis=-1))
            up = Unb @ val_nb.T
            gp = np.einsum("cqab,cqb->cqa", f["JinvT_nb"],
                           np.stack([Unb @ grad_nb[a].T for a in range(3)], axis=-1))
            up = np.where(interior[:, None], up, -um)
            gp = np.where(interior[:, None, None], gp, gm)
            nrm = f["normal"]
            jump = um - up
            v = f["sigma"][:, None] * jump - 0.5 * np.sum(nrm * (gm + gp), axis=-1)
            wv = -0.5 * jump[..., None] * nrm                              # physical vector
            wref = np.einsum("cqba,cqb->cqa", f["JinvT"], wv)              # J^-1 w
            JxW = f["JxW"]
            Y += (JxW * v) @ val
            for a in range(3):
                Y += (JxW * wref[..., a]) @ grad[a]
        return Y.reshape(-1)
