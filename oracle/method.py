"""Sparse-grid combination solve, its adjoint and the full-grid solve (oracle).

Test infrastructure only (see the package docstring).

Discrete problem of one component (paper eq. 9, algebraic form of Prop. 1):
unknown u_c[i,k] is the coefficient of psi_i(t) phi_k(x) (time index outer),

    S_c = A_{jt} (x) M_{jx} + B_{jt} (x) K_{jx},      S_c u_c = b_c,

    b_c[i,k] = sum_{n,m} W[i,n] (Phi^T M^J)[k,m] f[n,m]
               + psi_i'(0) (Phi^T M^J v0)[k] - g[i] (Phi^T K^J u0)[k],

with W, g as in ``timemat`` and Phi the nodal prolongation level jx -> J
(the data f, u0, v0 are nodal values on the finest grid, read as their
P1/Q1 interpolants in space and P1 interpolant in time; boundary values 0).

Combination (eq. 19) and lift (Sec. 2.1, the solution of (1) is u + u0):

    U[n,m] = u0[m] + sum_c s_c sum_{i,k} u_c[i,k] psi_i(t_n) phi_k(x_m).

S_c is factorised by SuperLU.  The discrete solution of long time levels is
sensitive to last-bit changes of the time-matrix entries, so the solve is
refined iteratively against the exact system: A and B are known to ~32
digits (hi + lo, see ``timemat.time_matrices_dd``), so is the 1-D stiffness
K (hi + lo, ``space.stiff_lo``: its zero row sums inside a block make the
low-frequency solution sensitive to last-bit changes of the diagonal), and
the residual b - S x is accumulated in double-double (``ddarith``).

The adjoint applies the explicit transposes of the three linear steps:
y_c = s_c Psi^T g Phi,  z_c = S_c^{-T} y_c,
df = sum_c W^T z_c (Phi^T M^J),  dv0 = sum_c (d0^T z_c)(Phi^T M^J),
du0 = sum_n g[n,:] - sum_c (g^T z_c)(Phi^T K^J).
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import ddarith, levels, space, timemat


class Problem:
    """The data of eq. (1) that fix the discrete operator.

    d in {1,2}; lengths: side lengths of Omega = prod (0, len_i);
    ncell, c_vals: piecewise-constant wave speed on a uniform block grid
    (x fastest); T: final time; L: sparse level (components C_L); b0:
    coarsest level of the combination (h_0 = 2^-b0, Sec. 6.3)."""

    def __init__(self, d, lengths, ncell, c_vals, T, L, b0=1):
        if d not in (1, 2) or len(lengths) != d or len(ncell) != d:
            raise ValueError("d must be 1 or 2 with one length/ncell per axis")
        if T <= 0 or L < 2:
            raise ValueError("need T > 0 and L >= 2")
        self.d = d
        self.T = float(T)
        self.L = int(L)
        self.b0 = int(b0)
        self.J = levels.finest_level(L)
        self.medium = space.Medium(lengths, ncell, c_vals)
        self.comps = levels.components(L, self.b0)
        self._cache = {}

    # ----- sizes -------------------------------------------------------
    @property
    def nt_fine(self):
        return 2 ** self.J + 1

    @property
    def ns_fine(self):
        return (2 ** self.J - 1) ** self.d

    def fine_shape(self):
        n = 2 ** self.J - 1
        return (self.nt_fine,) + (n,) * self.d

    # ----- cached operators --------------------------------------------
    def _get(self, key, make):
        if key not in self._cache:
            self._cache[key] = make()
        return self._cache[key]

    def mass(self, j):
        return self._get(("M", j), lambda: space.mass(j, self.medium))

    def stiff(self, j):
        return self._get(("K", j), lambda: space.stiff(j, self.medium))

    def stiff_lo(self, j):
        """Low parts of the stiffness entries (1-D), None in 2-D."""
        return self._get(("Klo", j), lambda: space.stiff_lo(j, self.medium))

    def phi(self, j, J=None):
        J = self.J if J is None else J
        return self._get(("Phi", j, J), lambda: space.interp(j, J, self.medium))

    def tmat(self, jt):
        """Time load vectors g, d0 of level jt."""
        def make():
            g, d0 = timemat.time_vectors(jt, self.T)
            return {"g": g, "d0": d0}
        return self._get(("T", jt), make)

    def tmat_dd(self, jt):
        """Double-double banded A, B of level jt (hi, lo parts)."""
        return self._get(("Tdd", jt), lambda: timemat.time_matrices_dd(jt, self.T))

    def wload(self, jt, J=None):
        J = self.J if J is None else J
        return self._get(("W", jt, J), lambda: timemat.load_weights(jt, J, self.T))

    def psi_nodes(self, jt, J=None):
        J = self.J if J is None else J
        return self._get(("Psi", jt, J), lambda: timemat.eval_at_nodes(jt, J, self.T))

    def cross_mass(self, jx):
        """(Phi^T M^J)[k,m] = (phi^J_m, phi^jx_k), exact by nesting."""
        return self._get(("MJc", jx), lambda: (self.phi(jx).T @ self.mass(self.J)).tocsr())

    def cross_stiff(self, jx):
        """(Phi^T K^J)[k,m] = (c^2 grad phi^J_m, grad phi^jx_k), exact by nesting
        (1-D: each entry evaluated exactly and rounded once)."""
        def make():
            if self.d == 1:
                return space.cross_stiff_1d(jx, self.J, self.medium)
            return (self.phi(jx).T @ self.stiff(self.J)).tocsr()
        return self._get(("KJc", jx), make)

    def time_sparse(self, jt, name):
        """High part of A or B of level jt as a sparse matrix."""
        band = self.tmat_dd(jt)[name + "_hi"]
        n = band.shape[0]
        return sp.diags([band[max(0, -(k - 2)):n - max(0, k - 2), k] for k in range(5)],
                        [k - 2 for k in range(5)], shape=(n, n), format="csr")

    def system(self, jx, jt):
        """Sparse S_c = A (x) M + B (x) K (time index outer), CSR (high parts)."""
        def make():
            return (sp.kron(self.time_sparse(jt, "A"), self.mass(jx))
                    + sp.kron(self.time_sparse(jt, "B"), self.stiff(jx))).tocsr()
        return self._get(("S", jx, jt), make)

    def factor(self, jx, jt):
        return self._get(("LU", jx, jt), lambda: spla.splu(self.system(jx, jt).tocsc()))

    # ----- the three linear steps --------------------------------------
    def load(self, jx, jt, f, u0, v0):
        """b_c of eq. (9) from nodal fine-grid data; shape (2^jt+1, n_space)."""
        f = np.asarray(f, dtype=np.float64).reshape(self.nt_fine, self.ns_fine)
        u0 = np.asarray(u0, dtype=np.float64).reshape(self.ns_fine)
        v0 = np.asarray(v0, dtype=np.float64).reshape(self.ns_fine)
        tm = self.tmat(jt)
        MJc = self.cross_mass(jx)
        b = self.wload(jt) @ np.asarray((MJc @ f.T).T)
        b += np.outer(tm["d0"], MJc @ v0)
        b -= np.outer(tm["g"], self.cross_stiff(jx) @ u0)
        return b

    def solve(self, jx, jt, b, transpose=False):
        """u = S_c^{-1} b (or S_c^{-T} b).  SuperLU of the high parts, then
        refinement with the residual formed in double-double from the exact
        time matrices (and, in 1-D, the exact stiffness entries) until the
        correction is below 1e-17 of the solution."""
        lu = self.factor(jx, jt)
        trans = "T" if transpose else "N"
        rhs = np.asarray(b, dtype=np.float64)
        shape = rhs.shape
        nt = 2 ** jt + 1
        rhs = rhs.reshape(nt, -1)
        x = lu.solve(rhs.reshape(-1), trans=trans).reshape(nt, -1)
        for _ in range(12):
            r = self._residual_dd(jx, jt, x, rhs, transpose)
            dx = lu.solve(r.reshape(-1), trans=trans).reshape(nt, -1)
            x = x + dx
            if np.abs(dx).max() <= 1e-17 * max(np.abs(x).max(), 1e-300):
                break
        return x.reshape(shape)

    def _padded(self, jx, which):
        """Rows of M or K as (cols, vals, vals_lo) padded to the longest row;
        vals_lo holds the low parts of K's entries in 1-D (else zeros)."""
        def make():
            A = (self.mass(jx) if which == "M" else self.stiff(jx)).tocsr()
            Alo = self.stiff_lo(jx) if which == "K" else None
            if Alo is not None:
                Alo = Alo.tocsr()
                assert (np.array_equal(Alo.indptr, A.indptr)
                        and np.array_equal(Alo.indices, A.indices))
            nnz = np.diff(A.indptr)
            width = int(nnz.max())
            cols = np.zeros((A.shape[0], width), dtype=np.int64)
            vals = np.zeros((A.shape[0], width))
            vlo = np.zeros((A.shape[0], width))
            for k in range(A.shape[0]):
                a, b = A.indptr[k], A.indptr[k + 1]
                cols[k, :b - a] = A.indices[a:b]
                vals[k, :b - a] = A.data[a:b]
                if Alo is not None:
                    vlo[k, :b - a] = Alo.data[a:b]
            return cols, vals, vlo
        return self._get(("pad", jx, which), make)

    def _residual_dd(self, jx, jt, X, Bv, transpose):
        """b - S x with S = A (x) M + B (x) K (or its transpose), every product
        and sum in double-double, A and B taken as hi + lo (and K too in 1-D,
        where its exact entries are known)."""
        dd = self.tmat_dd(jt)
        nt = X.shape[0]
        rh, rl = Bv.copy(), np.zeros_like(Bv)
        for tname, sname in (("A", "M"), ("B", "K")):
            cols, vals, vlo = self._padded(jx, sname)   # M, K are symmetric
            Yh, Yl = ddarith.zeros(X.shape)
            for slot in range(cols.shape[1]):
                xs = X[:, cols[:, slot]]
                ph, pl = ddarith.two_prod(xs, vals[None, :, slot])
                Yh, Yl = ddarith.add(Yh, Yl, ph, pl)
                Yh, Yl = ddarith.add(Yh, Yl, xs * vlo[None, :, slot], 0.0)
            Th, Tl = dd[tname + "_hi"], dd[tname + "_lo"]
            for k in range(5):
                off = k - 2
                i = np.arange(max(0, -off), min(nt, nt - off))
                if transpose:
                    # (A^T)[i, i+off] = A[i+off, i] = band[i+off, 2-off]
                    ah = Th[i + off, 2 - off][:, None]
                    al = Tl[i + off, 2 - off][:, None]
                else:
                    ah = Th[i, k][:, None]
                    al = Tl[i, k][:, None]
                ph, pl = ddarith.mul(ah, al, Yh[i + off], Yl[i + off])
                sh, sl = ddarith.add(rh[i], rl[i], -ph, -pl)
                rh[i], rl[i] = sh, sl
        return rh + rl

    def prolong(self, jx, jt, u):
        """Nodal values on the finest grid of sum_{i,k} u[i,k] psi_i phi_k."""
        Y = self.psi_nodes(jt) @ u                    # (NT, n_space(jx))
        return np.asarray((self.phi(jx) @ Y.T).T)     # (NT, NS)

    # ----- forward / adjoint -------------------------------------------
    def component_solutions(self, f, u0, v0):
        return [self.solve(jx, jt, self.load(jx, jt, f, u0, v0))
                for jx, jt, _ in self.comps]

    def combine(self, sols, u0):
        U = np.tile(np.asarray(u0, dtype=np.float64).reshape(1, self.ns_fine),
                    (self.nt_fine, 1))
        for (jx, jt, s), u in zip(self.comps, sols):
            U += s * self.prolong(jx, jt, u)
        return U

    def forward(self, f, u0, v0):
        """U on the finest grid, shape (2^J+1, n^d) flattened in space."""
        return self.combine(self.component_solutions(f, u0, v0), u0)

    def adjoint(self, g):
        """(df, du0, dv0) = F^T g for the linear map F: (f,u0,v0) -> U."""
        g = np.asarray(g, dtype=np.float64).reshape(self.nt_fine, self.ns_fine)
        df = np.zeros_like(g)
        du0 = g.sum(axis=0)
        dv0 = np.zeros(self.ns_fine)
        for jx, jt, s in self.comps:
            y = s * (self.psi_nodes(jt).T @ np.asarray((self.phi(jx).T @ g.T).T))
            z = self.solve(jx, jt, y, transpose=True)
            tm = self.tmat(jt)
            MJc = self.cross_mass(jx)
            df += np.asarray((MJc.T @ (self.wload(jt).T @ z).T).T)
            dv0 += MJc.T @ (tm["d0"] @ z)
            du0 -= self.cross_stiff(jx).T @ (tm["g"] @ z)
        return df, du0, dv0

    def full_grid(self, j, f, u0, v0):
        """P_{j,j} (eq. 10 with jx = jt = j <= J) plus u0, on the finest grid."""
        u = self.solve(j, j, self.load(j, j, f, u0, v0))
        U = np.tile(np.asarray(u0, dtype=np.float64).reshape(1, self.ns_fine),
                    (self.nt_fine, 1))
        return U + self.prolong(j, j, u)


# ----------------------------------------------------------------------
# Extras used only by the convergence-rate pins: the load of eq. (9) built
# from closed-form data by quadrature (so that only the discretisation error
# is measured), and the L^2(Q_T) error of the combined solution.
# ----------------------------------------------------------------------

_NQ = 5
_QX, _QW = np.polynomial.legendre.leggauss(_NQ)


def fine_quadrature(J, length, nq=_NQ):
    """Gauss points/weights (nq per element) on every element of the level-J
    mesh of (0,length)."""
    qx, qw = (_QX, _QW) if nq == _NQ else np.polynomial.legendre.leggauss(nq)
    h = length / 2 ** J
    left = h * np.arange(2 ** J)
    pts = (left[:, None] + 0.5 * h * (qx[None, :] + 1.0)).reshape(-1)
    wts = np.tile(0.5 * h * qw, 2 ** J)
    return pts, wts


def load_exact(prob, jx, jt, f_fn, u0_fn, v0_fn, grad_u0_fn):
    """b_c of eq. (9) for closed-form data, by quadrature on the finest mesh.

    f_fn(t, *x) and the initial data are vectorised callables on tensor grids;
    grad_u0_fn returns the list of partial derivatives.  Only c == const
    problems use this (c^2 is taken from block 0)."""
    from . import basis
    J = prob.J
    T = prob.T
    c2 = float(prob.medium.c.reshape(-1)[0]) ** 2
    tq, tw = fine_quadrature(J, T)
    dpsi = basis.time_basis(jt, T, tq, 1) * (tw * np.exp(-tq / T))[:, None]
    d0 = basis.time_basis(jt, T, np.array([0.0]), 1)[0]
    g = dpsi.sum(axis=0)
    axes = []
    for ax in range(prob.d):
        xq, xw = fine_quadrature(J, prob.medium.lengths[ax])
        axes.append((xq, xw, basis.hat_1d(jx, prob.medium.lengths[ax], xq),
                     basis.hat_1d_deriv(jx, prob.medium.lengths[ax], xq)))
    if prob.d == 1:
        xq, xw, ph, dph = axes[0]
        F = f_fn(tq[:, None], xq[None, :])                      # (t, x)
        b = dpsi.T @ (F @ (ph * xw[:, None]))
        b += np.outer(d0, (v0_fn(xq) * xw) @ ph)
        (du,) = grad_u0_fn(xq)
        b -= np.outer(g, c2 * (du * xw) @ dph)
        return b
    (xq, xw, phx, dphx), (yq, yw, phy, dphy) = axes
    F = f_fn(tq[:, None, None], xq[None, None, :], yq[None, :, None])  # (t,y,x)
    P = np.einsum("tyx,xk->tyk", F, phx * xw[:, None])
    P = np.einsum("tyk,yl->tlk", P, phy * yw[:, None])
    b = np.einsum("ti,tlk->ilk", dpsi, P).reshape(dpsi.shape[1], -1)
    V = v0_fn(xq[None, :], yq[:, None]) * yw[:, None] * xw[None, :]
    b += np.outer(d0, (phy.T @ V @ phx).reshape(-1))
    ux, uy = grad_u0_fn(xq[None, :], yq[:, None])
    W2 = yw[:, None] * xw[None, :]
    Ku0 = phy.T @ (c2 * ux * W2) @ dphx + dphy.T @ (c2 * uy * W2) @ phx
    b -= np.outer(g, Ku0.reshape(-1))
    return b


def combined_at(prob, sols, tq, xqs, u0_fn=None):
    """Combined solution sum_c s_c u_c(x,t) (+ u0) on a tensor grid of points."""
    from . import basis
    out = 0.0
    for (jx, jt, s), u in zip(prob.comps, sols):
        Pt = basis.time_basis(jt, prob.T, tq, 0)
        if prob.d == 1:
            Px = basis.hat_1d(jx, prob.medium.lengths[0], xqs[0])
            out = out + s * (Pt @ u @ Px.T)
        else:
            Px = basis.hat_1d(jx, prob.medium.lengths[0], xqs[0])
            Py = basis.hat_1d(jx, prob.medium.lengths[1], xqs[1])
            n = 2 ** jx - 1
            V = np.einsum("ti,iyx->tyx", Pt, u.reshape(-1, n, n))
            V = np.einsum("tyx,qx->tyq", V, Px)
            out = out + s * np.einsum("tyq,py->tpq", V, Py)
    if u0_fn is not None:
        if prob.d == 1:
            out = out + u0_fn(xqs[0])[None, :]
        else:
            out = out + u0_fn(xqs[0][None, :], xqs[1][:, None])[None, :, :]
    return out


def solution_at(prob, sols, u0, times, deriv=0):
    """Nodal values on the finest grid of u_h(t) = u0 + sum_c s_c u_c(., t)
    (deriv = 0) or of d_t u_h(t) (deriv = 1) at the instants ``times``, shape
    (len(times), n^d).  Spline values/derivatives at arbitrary t from the
    B-spline recursion, the nested spatial prolongation Phi_{jx -> J}."""
    from . import basis
    t = np.atleast_1d(np.asarray(times, dtype=np.float64))
    out = np.zeros((t.size, prob.ns_fine))
    if deriv == 0:
        out += np.asarray(u0, dtype=np.float64).reshape(1, prob.ns_fine)
    for (jx, jt, s), u in zip(prob.comps, sols):
        Pt = basis.time_basis(jt, prob.T, t, deriv)           # (K, n_time)
        uc = np.asarray(u).reshape(Pt.shape[1], -1)            # (n_time, n_space)
        P = space.interp(jx, prob.J, prob.medium)              # (NS, n_space)
        out += s * np.asarray((P @ (Pt @ uc).T).T)
    return out


def energy(prob, sols, u0, times):
    """Energy of the computed solution at the given instants (Sec. 6.3):

        E(t) = 1/2 ||d_t u_h(t)||^2 + 1/2 ||c grad u_h(t)||^2,

    u_h = u0 + sum_c s_c u_c the lifted combination solution.  For fixed t,
    u_h(t) and d_t u_h(t) are P1/Q1 functions on the finest mesh (the spaces
    are nested), so with their nodal values w and v the integrals are exactly
    1/2 v^T M_J v + 1/2 w^T K_J w (K_J exact in c^2; hi + lo in 1-D)."""
    W = solution_at(prob, sols, u0, times, 0)
    V = solution_at(prob, sols, u0, times, 1)
    M = space.mass(prob.J, prob.medium)
    K = space.stiff(prob.J, prob.medium)
    Klo = space.stiff_lo(prob.J, prob.medium)
    KW = np.asarray((K @ W.T).T)
    if Klo is not None:
        KW = KW + np.asarray((Klo @ W.T).T)
    MV = np.asarray((M @ V.T).T)
    return 0.5 * np.sum(V * MV, axis=1) + 0.5 * np.sum(W * KW, axis=1)


def l2_error(prob, sols, u_fn, u0_fn=None, comps=None):
    """(||u - u_h||, ||u||) in L^2(Q_T) by Gauss quadrature on the finest mesh.

    sols/comps: component solutions and their (jx, jt, sign) list (default:
    the problem's components)."""
    saved = prob.comps
    if comps is not None:
        prob.comps = comps
    try:
        J = prob.J
        tq, tw = fine_quadrature(J, prob.T)
        xs = [fine_quadrature(J, prob.medium.lengths[a]) for a in range(prob.d)]
        uh = combined_at(prob, sols, tq, [x[0] for x in xs], u0_fn)
    finally:
        prob.comps = saved
    if prob.d == 1:
        ue = u_fn(tq[:, None], xs[0][0][None, :])
        W = tw[:, None] * xs[0][1][None, :]
    else:
        ue = u_fn(tq[:, None, None], xs[0][0][None, None, :], xs[1][0][None, :, None])
        W = tw[:, None, None] * xs[1][1][None, :, None] * xs[0][1][None, None, :]
    return np.sqrt(np.sum(W * (ue - uh) ** 2)), np.sqrt(np.sum(W * ue ** 2))


def l2_error_rule(prob, sols, u0, u_fn, nq_t=3, nq_x=2):
    """(int (u - u_h)^2, int u^2) over Q_T by the tensor Gauss rule with nq_t
    points per finest time interval and nq_x points per finest element along
    each space axis (Sec. 6.3 reports relative L^2(Q_T) errors); u_h = I_J u0
    + sum_c s_c u_c with the nodal u0 read as its finest-grid interpolant, as
    the solver reads it.  u_fn(t, x) or u_fn(t, x, y), vectorised."""
    from . import basis
    J = prob.J
    tq, tw = fine_quadrature(J, prob.T, nq_t)
    xs = [fine_quadrature(J, prob.medium.lengths[a], nq_x) for a in range(prob.d)]
    uh = combined_at(prob, sols, tq, [x[0] for x in xs])
    P = [basis.hat_1d(J, prob.medium.lengths[a], xs[a][0]) for a in range(prob.d)]
    u0 = np.asarray(u0, dtype=np.float64)
    if prob.d == 1:
        lift = P[0] @ u0.reshape(-1)
        ue = u_fn(tq[:, None], xs[0][0][None, :])
        W = tw[:, None] * xs[0][1][None, :]
    else:
        n = 2 ** J - 1
        lift = P[1] @ u0.reshape(n, n) @ P[0].T                # (y, x)
        ue = u_fn(tq[:, None, None], xs[0][0][None, None, :], xs[1][0][None, :, None])
        W = tw[:, None, None] * xs[1][1][None, :, None] * xs[0][1][None, None, :]
    uh = uh + lift[None]
    return float(np.sum(W * (ue - uh) ** 2)), float(np.sum(W * ue ** 2))

