"""The ADER-AFE-DG step, written plainly in float64 (Sec. 4.2 - 4.5).

Notation: cell i has sub-tets k with sub-tet node -> cell DOF map P_k (conn),
|J_k| = |det J_k|, G_k = J_k^{-1}; reference matrices M^, K^_d, V^_d = K^_d^T,
D^_d, Z^; time basis on N+1 Gauss-Legendre nodes tau_a with weights w_a.

Readings taken where the paper is silent, garbled or inconsistent:

R1 (assembly, Sec. 4.3-4.4): |P_i| printed in front of the sums of reference
   integrals (K_t,i, K_1,i, M_i) is read as the sub-tet Jacobian weighting of
   each term, X_i = sum_k |J_k| P_k^T X^ P_k, which is what the sum over
   sub-tets with the Jacobian (eq:ader2) produces.
R2 (time basis): N+1 Gauss-Legendre nodes; then M_tau = diag(w), the space-time
   K_1,i = K_tau (x) M_i and the spatial stiffness is M_tau (x) K^_d, so
   K_1,i^{-1} = K_tau^{-1} (x) M_i^{-1}.  Because K_tau 1 = psi(0), the F_0 term
   gives u^n at every time node, and eq:ader4 becomes
       q[b] = u^n - sum_a (K_tau^{-1})_{ba} M_i^{-1} R[a](q),
       R[a] = w_a sum_k P_k^T |J_k| sum_d K^_d f*_{d,k}[a],
   with the contravariant nodal flux f*_d = dt sum_x G_k[d, x] F_x(q, grad q).
R3 (iteration, eq:ader4): the predictor is the fixed point of that map.  It is
   reached by Anderson acceleration of the same map with depth m (m = 0 is
   the plain fixed-point iteration of the paper), starting from q = u^n, and
   stops when max|G(q) - q| <= tol * max(1, max|G(q)|); the result is G(q).
   tol = 0 asks for exactly max_iter applications of the map (the same
   sweeps on both sides of a parity check), which counts as converged.
R4 (time integrals, eqn.TAvectors): f* already holds dt, so the volume term
   uses F*bar_d = sum_a w_a f*_d[a]; the face flux uses the physical
   Fbar = dt sum_a w_a F(q[a]) and qbar = dt sum_a w_a q[a].
R5 (faces, Sec. 4.4): the sum over faces runs over the cell's boundary
   sub-triangles; each integral is 2 A_t Z^ (reference triangle area 1/2).
   In the Rusanov flux "+" is the neighbour and "-" this cell, n outward;
   |lambda_max| is the largest |v.n| + c over the triangle's face nodes on both
   sides from qbar/dt and |lambda^v_max| the largest viscous eigenvalue
   max(4 mu/(3 rho), kappa/(c_v rho)) likewise with each side's viscosity;
   one value per sub-triangle.
R6 (detector, Sec. 4.5): the divergence is the face integral of the velocity
   jump over the cell volume; it enters the flattener multiplied by the cell
   diameter h_i (undivided form) so that it compares with m1 c; c_min is the
   minimum sound speed over the face nodes on both sides; states are u^n.
R7 (artificial viscosity, Sec. 4.5, text ends before the formula):
   mu_i = mu + beta_i * rho_i * lambda_i * h_s, h_s = h_i / (2N+1), with rho_i
   the cell-mean density and lambda_i the largest nodal |v| + c, i.e. the
   viscosity for which the mesh Reynolds number is one, scaled by beta_i.
R8 (time step, eqn.timestep): h_i = cell diameter; the max runs over all DOFs
   with h inside it taken per cell, lambda^v = max(4 mu_i / (3 rho),
   kappa / (c_v rho)).
R9 (initial data): nodal interpolation of the primitive variables, converted
   to conserved variables.
R15 (heat conduction, Sec. 2): kappa is a constant of the simulation, not
   raised with the artificial viscosity of R7; T = p / (rho R) with
   R = (gamma - 1) c_v (c_v a parameter, 2.5 as in the paper's viscous test);
   the second viscous eigenvalue gamma mu / (Pr rho) with Pr = mu gamma c_v /
   kappa is kappa / (c_v rho).
R21 (Dirichlet boundaries, Sec. 5.1-5.2 "Dirichlet boundary conditions on all
   sides" with the exact solution): on a bounded mesh a boundary sub-triangle
   takes as its "+" side the exact solution at its face nodes' positions at
   the predictor's time nodes t^n + tau_a dt, so qbar+ = dt sum_a w_a q_e(a)
   and Fbar+ = dt sum_a w_a F(q_e(a)); the Rusanov flux of R5 is then taken
   as at an interior triangle, with the "+" wave speeds from qbar+ / dt.  The
   detector (R6) counts no velocity jump and no outside sound speed across a
   boundary triangle.  With viscosity or heat conduction the "+" flux is the
   Navier-Stokes flux of the exact state with the exact solution's gradient
   (given with the data) and the inside cell's viscosity; the penalty of R5
   takes the inside cell's viscosity and length scale on both sides.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import cho_factor, cho_solve

from .physics import flux, max_eig, prim_to_cons, pressure, sound_speed, visc_eig
from .refelem import ref_element, time_basis
from .subgrid import build_cells, faces_of_cells


@dataclass
class Params:
    gamma: float = 1.4
    mu: float = 0.0
    kappa: float = 0.0  # heat conduction coefficient (R15)
    cv: float = 2.5     # specific heat at constant volume: R = (gamma - 1) c_v
    m1: float = 0.1
    av: bool = False
    tol: float = 1e-12
    max_iter: int = 300
    depth: int = 63


@dataclass
class StepReport:
    iters: dict = field(default_factory=dict)
    converged: bool = True
    positive: bool = True
    mu: dict = field(default_factory=dict)
    beta: dict = field(default_factory=dict)
    pred: dict = field(default_factory=dict)
    ti: dict = field(default_factory=dict)


def dof_counts(mesh: dict, N: int) -> np.ndarray:
    """Number of cell DOFs from the sub-grid's entity counts.

    Sub-grid of a cell with V vertices, F faces and E polygon edges: V + F + 1
    vertices, 3E + V + F edges, 5E triangles, 2E sub-tets; a P_N Lagrange space
    has N-1 nodes inside each edge, (N-1)(N-2)/2 inside each triangle and
    (N-1)(N-2)(N-3)/6 inside each tet.
    """
    n = mesh["n_cells"]
    fp = mesh["face_ptr"]
    V = np.zeros(n, dtype=np.int64)
    F = np.zeros(n, dtype=np.int64)
    E = np.zeros(n, dtype=np.int64)
    verts = [set() for _ in range(n)]
    for f, cells in enumerate(mesh["face_cell"]):
        k = int(fp[f + 1] - fp[f])
        for c in cells:
            if c < 0:  # boundary face: one cell only
                continue
            F[c] += 1
            E[c] += k
            verts[c].update(int(v) for v in mesh["face_vtx"][fp[f]:fp[f + 1]])
    E //= 2
    V[:] = [len(s) for s in verts]
    a = N - 1
    return (V + F + 1) + a * (3 * E + V + F) + (a * (a - 1) // 2) * 5 * E + (a * (a - 1) * (a - 2) // 6) * 2 * E


class Oracle:
    """Plain implementation of one ADER-AFE-DG step on a periodic mesh.

    State layout (same as the library's): SoA u[5, ndof] in cell-major order,
    cell c owning u[:, dof_ptr[c]:dof_ptr[c+1]] in the cell's DOF numbering.
    `cells` restricts the outputs to a subset (their neighbours, and second
    neighbours when artificial viscosity is on, are built as needed).
    """

    def __init__(self, mesh: dict, N: int, params: Params = Params(), cells=None, boundary=None,
                 boundary_grad=None):
        self.mesh = mesh
        self.N = N
        self.p = params
        # exact solution for the Dirichlet data of a bounded mesh (R21):
        # boundary(x [n, 3], t) -> primitive (rho, u, v, w, p) [n, 5]; with
        # viscosity or heat conduction also boundary_grad(x, t) -> its
        # gradient [n, 3, 5], [.., d, k] = d prim_k / d x_d
        self.bounded = bool(mesh.get("bounded", False))
        self.boundary = boundary
        self.boundary_grad = boundary_grad
        self.t = 0.0
        self.ref = ref_element(N)
        self.tb = time_basis(N)
        n = mesh["n_cells"]
        self.n_cells = n
        counts = dof_counts(mesh, N)
        self.dof_ptr = np.concatenate([[0], np.cumsum(counts)])
        self.ndof = int(self.dof_ptr[-1])
        cf = faces_of_cells(mesh)
        self.targets = list(range(n)) if cells is None else sorted(set(int(c) for c in cells))
        paired = set(self.targets)
        if params.av and cells is not None:
            for c in self.targets:
                for f, side in cf[c]:
                    if mesh["face_cell"][f][1 - side] >= 0:
                        paired.add(int(mesh["face_cell"][f][1 - side]))
        self.paired = sorted(paired)
        self.grids = build_cells(mesh, N, self.paired)
        for c, g in self.grids.items():
            if g.ndof != counts[c]:
                raise AssertionError("DOF count mismatch")
        self._chol = {}
        self._mass = {}

    # ------------------------------------------------------------------ helpers
    def cell_state(self, u: np.ndarray, c: int) -> np.ndarray:
        """[ndof_c, 5] view-copy of cell c's DOFs."""
        return u[:, self.dof_ptr[c]:self.dof_ptr[c + 1]].T.copy()

    def mass(self, c: int) -> np.ndarray:
        """M_i = sum_k |J_k| P_k^T M^ P_k (R1)."""
        if c not in self._mass:
            g = self.grids[c]
            M = np.zeros((g.ndof, g.ndof))
            for k in range(len(g.conn)):
                idx = g.conn[k]
                M[np.ix_(idx, idx)] += g.detJ[k] * self.ref.M_f
            self._mass[c] = M
        return self._mass[c]

    def mass_solve(self, c: int, rhs: np.ndarray) -> np.ndarray:
        if c not in self._chol:
            self._chol[c] = cho_factor(self.mass(c), lower=True)
        return cho_solve(self._chol[c], rhs)

    def dof_coords(self) -> np.ndarray:
        """[3, ndof] DOF coordinates in each cell's frame (targets only filled)."""
        x = np.full((3, self.ndof), np.nan)
        for c in self.targets:
            x[:, self.dof_ptr[c]:self.dof_ptr[c + 1]] = self.grids[c].dof_x.T
        return x

    def initial_state(self, field_fn) -> np.ndarray:
        """Nodal interpolation of primitive variables (R9), for every built cell."""
        u = np.zeros((5, self.ndof))
        L = self.mesh["box"]
        for c, g in self.grids.items():
            w = field_fn(g.dof_x if self.bounded else np.mod(g.dof_x, L))
            u[:, self.dof_ptr[c]:self.dof_ptr[c + 1]] = prim_to_cons(w, self.p.gamma).T
        return u

    # ------------------------------------------------------------ detector / AV
    def detector(self, u: np.ndarray, c: int):
        """beta_i and mu_i of cell c from u^n (Sec. 4.5, R6, R7)."""
        g = self.grids[c]
        gam = self.p.gamma
        N = self.N
        uc = self.cell_state(u, c)
        zrow = self.ref.Z_f.sum(axis=0)  # int_tri phi_j
        jump_int = 0.0
        cmin = math.inf
        for k in range(len(g.conn)):
            qi = uc[g.face_dof[k]]
            if g.nbr[k] < 0:  # boundary triangle: no jump, inside sound speed only (R21)
                cmin = min(cmin, float(sound_speed(qi, gam).min()))
                continue
            qo = self.cell_state(u, int(g.nbr[k]))[g.nbr_face_dof[k]]
            vi = qi[:, 1:4] / qi[:, :1]
            vo = qo[:, 1:4] / qo[:, :1]
            jn = (vo - vi) @ g.tri_normal[k]
            jump_int += 2.0 * g.tri_area[k] * float(zrow @ jn)
            cmin = min(cmin, float(sound_speed(qi, gam).min()), float(sound_speed(qo, gam).min()))
        vol = g.volume
        div = jump_int / vol
        m1 = self.p.m1
        beta = min(1.0, max(0.0, -(g.h * div + m1 * cmin) / (m1 * cmin)))
        if not self.p.av:
            return 0.0, self.p.mu
        rho_mean = float(self.mass(c).sum(axis=0) @ uc[:, 0]) / vol
        lam = float(max_eig(uc, gam).max())
        mu_c = self.p.mu + beta * rho_mean * lam * g.h / (2 * N + 1)
        return beta, mu_c

    def viscosities(self, u: np.ndarray, cells) -> dict:
        out = {}
        for c in cells:
            out[c] = self.detector(u, c)[1] if self.p.av else self.p.mu
        return out

    def cfl_dt(self, u: np.ndarray, cfl: float) -> float:
        """Time step of eqn.timestep (R8) over the target cells."""
        N = self.N
        mus = self.viscosities(u, self.targets)
        hmin = min(self.grids[c].h for c in self.targets)
        smax = 0.0
        for c in self.targets:
            g = self.grids[c]
            uc = self.cell_state(u, c)
            lam = max_eig(uc, self.p.gamma) + 2.0 * visc_eig(uc, mus[c], self.p.kappa, self.p.cv) * (2 * N + 1) / g.h
            smax = max(smax, float(lam.max()))
        return cfl * hmin / ((2 * N + 1) * smax)

    # --------------------------------------------------------------- predictor
    def _nodal_flux(self, c: int, q: np.ndarray, mu: float):
        """Physical flux at every sub-tet node and time node: [A, K, P, 3, 5]."""
        g = self.grids[c]
        qk = q[:, g.conn, :]  # [A, K, P, 5]
        grad = None
        if mu != 0.0 or self.p.kappa != 0.0:
            # grad q at node m of sub-tet k: sum_d G_k[d, x] (D^_d q_k)_m
            ref_grad = np.einsum("dml,aklv->akmdv", self.ref.D_f, qk)
            grad = np.einsum("kdx,akmdv->akmxv", g.G, ref_grad)
        return flux(qk, self.p.gamma, mu, grad, self.p.kappa, self.p.cv)

    def _contravariant(self, c: int, F: np.ndarray, dt: float) -> np.ndarray:
        """f*_d = dt sum_x G_k[d, x] F_x  (eq:modified_fluxes): [A, K, P, 3, 5]."""
        return dt * np.einsum("kdx,akpxv->akpdv", self.grids[c].G, F)

    def predictor_map(self, c: int, q: np.ndarray, un: np.ndarray, dt: float, mu: float) -> np.ndarray:
        """One application of eq:ader4 (R2): q [A, ndof, 5] -> [A, ndof, 5]."""
        g = self.grids[c]
        A = self.tb.nt
        fstar = self._contravariant(c, self._nodal_flux(c, q, mu), dt)
        # r_k[a] = w_a |J_k| sum_d K^_d f*_d  ->  [A, K, P, 5]
        r = np.einsum("a,k,dmp,akpdv->akmv", self.tb.w, g.detJ, self.ref.K_f, fstar)
        Rg = np.zeros((A, g.ndof, 5))
        for a in range(A):
            np.add.at(Rg[a], g.conn, r[a])
        S = self.mass_solve(c, Rg.transpose(1, 0, 2).reshape(g.ndof, A * 5))
        S = S.reshape(g.ndof, A, 5).transpose(1, 0, 2)
        return un[None, :, :] - np.einsum("ba,anv->bnv", self.tb.K_tau_inv, S)

    def predictor(self, c: int, un: np.ndarray, dt: float, mu: float, depth=None, tol=None, max_iter=None):
        """Fixed point of eq:ader4 by Anderson(depth) iteration (R3).

        Returns (q [A, ndof, 5], iterations, converged)."""
        depth = self.p.depth if depth is None else depth
        tol = self.p.tol if tol is None else tol
        max_iter = self.p.max_iter if max_iter is None else max_iter
        A = self.tb.nt
        x = np.broadcast_to(un, (A,) + un.shape).copy()
        Fh, Gh = [], []
        for it in range(max_iter):
            gx = self.predictor_map(c, x, un, dt, mu)
            f = gx - x
            if np.abs(f).max() <= tol * max(1.0, np.abs(gx).max()):
                return gx, it + 1, True
            if depth == 0:
                x = gx
                continue
            Fh.append(f.ravel())
            Gh.append(gx.ravel())
            if len(Fh) > depth + 1:
                Fh.pop(0)
                Gh.pop(0)
            if len(Fh) == 1:
                x = gx
                continue
            dF = np.diff(np.array(Fh), axis=0).T
            dG = np.diff(np.array(Gh), axis=0).T
            gam, *_ = np.linalg.lstsq(dF, f.ravel(), rcond=None)
            x = (gx.ravel() - dG @ gam).reshape(gx.shape)
        return gx, max_iter, tol == 0.0

    def time_integrals(self, c: int, q: np.ndarray, dt: float, mu: float):
        """qbar, volume term and face traces from the converged predictor (R4).

        Returns dict with
            qbar   [ndof, 5]          dt sum_a w_a q[a]
            vol    [ndof, 5]          sum_k P_k^T |J_k| sum_d V^_d F*bar_{d,k}
            tq     [K, nf, 5]         qbar at each boundary triangle's nodes
            tF     [K, nf, 3, 5]      dt sum_a w_a F(q[a]) there (sub-tet k's gradient)
        """
        g = self.grids[c]
        w = self.tb.w
        F = self._nodal_flux(c, q, mu)
        fstar = self._contravariant(c, F, dt)
        fbar = np.einsum("a,akpdv->kpdv", w, fstar)
        vk = np.einsum("k,dpm,kmdv->kpv", g.detJ, self.ref.V_f, fbar)
        vol = np.zeros((g.ndof, 5))
        np.add.at(vol, g.conn, vk)
        qbar = dt * np.einsum("a,anv->nv", w, q)
        fn = self.ref.face_nodes_a
        tq = qbar[g.face_dof]
        tF = dt * np.einsum("a,akjxv->kjxv", w, F[:, :, fn])
        return dict(qbar=qbar, vol=vol, tq=tq, tF=tF)

    # --------------------------------------------------------------- corrector
    def rusanov(self, c: int, k: int, ti: dict, mus: dict, dt: float) -> np.ndarray:
        """Time-integrated Rusanov flux G [nf, 5] at the nodes of cell c's boundary
        triangle k, eq. (3.33) with the readings R4-R5."""
        g = self.grids[c]
        gam = self.p.gamma
        N = self.N
        nb = int(g.nbr[k])
        qi, Fi = ti[c]["tq"][k], ti[c]["tF"][k]
        if nb < 0:
            qo, Fo = self.boundary_traces(c, k, dt, mus[c])
            nb = c  # viscosity and length scale of the inside (R21)
        else:
            kn = int(g.nbr_tri[k])
            perm = g.nbr_perm[k]
            qo, Fo = ti[nb]["tq"][kn][perm], ti[nb]["tF"][kn][perm]
        n = g.tri_normal[k]
        wi, wo = qi / dt, qo / dt
        vi = wi[:, 1:4] / wi[:, :1]
        vo = wo[:, 1:4] / wo[:, :1]
        lam = max(float((np.abs(vi @ n) + sound_speed(wi, gam)).max()),
                  float((np.abs(vo @ n) + sound_speed(wo, gam)).max()))
        kap, cv = self.p.kappa, self.p.cv
        lamv = max(float(visc_eig(wi, mus[c], kap, cv).max()), float(visc_eig(wo, mus[nb], kap, cv).max()))
        eps = (2 * N + 1) / ((g.h + self.grids[nb].h) * math.sqrt(math.pi / 2.0))
        s = lam + 2.0 * eps * lamv
        return 0.5 * np.einsum("jxv,x->jv", Fo + Fi, n) - 0.5 * s * (qo - qi)

    def boundary_traces(self, c: int, k: int, dt: float, mu: float = 0.0):
        """qbar+ [nf, 5] and Fbar+ [nf, 3, 5] of the exact solution at the face
        nodes of cell c's boundary triangle k over the step (R21); mu is the
        inside cell's viscosity."""
        if self.boundary is None:
            raise ValueError("a bounded mesh needs the exact solution for its boundary data")
        g = self.grids[c]
        x = g.dof_x[g.face_dof[k]]
        gam = self.p.gamma
        viscous = mu != 0.0 or self.p.kappa != 0.0
        if viscous and self.boundary_grad is None:
            raise ValueError("viscous boundary data need the exact solution's gradient")
        qs, Fs = [], []
        for tau in self.tb.tau:
            t = self.t + tau * dt
            w = self.boundary(x, t)
            q = prim_to_cons(w, gam)
            gq = None
            if viscous:
                # d(conserved)/dx from d(primitive)/dx: rho, rho v, rho E = p/(gamma-1) + rho |v|^2 / 2
                gw = self.boundary_grad(x, t)  # [nf, 3, 5]
                rho, vel = w[:, 0], w[:, 1:4]
                gq = np.empty_like(gw)
                gq[..., 0] = gw[..., 0]
                gq[..., 1:4] = vel[:, None, :] * gw[..., :1] + rho[:, None, None] * gw[..., 1:4]
                gq[..., 4] = (gw[..., 4] / (gam - 1.0) + 0.5 * (vel * vel).sum(-1)[:, None] * gw[..., 0]
                              + rho[:, None] * np.einsum("ni,ndi->nd", vel, gw[..., 1:4]))
            qs.append(q)
            Fs.append(flux(q, gam, mu, gq, self.p.kappa, self.p.cv))
        qa, Fa = np.stack(qs), np.stack(Fs)
        qbar = dt * np.einsum("a,ajv->jv", self.tb.w, qa)
        Fbar = dt * np.einsum("a,ajxv->jxv", self.tb.w, Fa)
        return qbar, Fbar

    def face_term(self, c: int, ti: dict, mus: dict, dt: float) -> np.ndarray:
        """sum_t P_t^T 2 A_t Z^ G_t (R5)."""
        g = self.grids[c]
        out = np.zeros((g.ndof, 5))
        for k in range(len(g.conn)):
            Gf = self.rusanov(c, k, ti, mus, dt)
            np.add.at(out, g.face_dof[k], 2.0 * g.tri_area[k] * (self.ref.Z_f @ Gf))
        return out

    # -------------------------------------------------------------------- step
    def ring(self) -> list:
        """Target cells and their face neighbours."""
        ring = set(self.targets)
        for c in self.targets:
            ring.update(int(x) for x in self.grids[c].nbr if x >= 0)
        return sorted(ring)

    def step(self, u: np.ndarray, dt: float, depth=None, tol=None, max_iter=None, keep=False, t: float = 0.0):
        """One ADER step from time t: detector, predictor, corrector, positivity
        check.  Returns (u_new, report); only target cells of u_new are updated.
        keep=True also stores the predictor results in report.pred / report.ti.
        t matters only for the boundary data of a bounded mesh (R21)."""
        self.t = float(t)
        rep = StepReport()
        ring = self.ring()
        mus = {}
        for c in ring:
            if self.p.av:
                beta, mu_c = self.detector(u, c)
            else:
                beta, mu_c = 0.0, self.p.mu
            mus[c] = mu_c
            rep.beta[c] = beta
        rep.mu = mus
        ti = {}
        for c in ring:
            un = self.cell_state(u, c)
            q, it, ok = self.predictor(c, un, dt, mus[c], depth, tol, max_iter)
            rep.iters[c] = it
            rep.converged &= ok
            ti[c] = self.time_integrals(c, q, dt, mus[c])
            if keep:
                rep.pred[c] = q
        if keep:
            rep.ti = ti
        unew = u.copy()
        for c in self.targets:
            rhs = ti[c]["vol"] - self.face_term(c, ti, mus, dt)
            du = self.mass_solve(c, rhs)
            newc = self.cell_state(u, c) + du
            unew[:, self.dof_ptr[c]:self.dof_ptr[c + 1]] = newc.T
            ok = bool(np.all(np.isfinite(newc)) and np.all(newc[:, 0] > 0) and np.all(pressure(newc, self.p.gamma) > 0))
            rep.positive &= ok
        return unew, rep

    # ----------------------------------------------------------------- metrics
    def l2_error(self, u: np.ndarray, exact_fn, var: int = 0, qorder_pts=None) -> float:
        """(sum_cells int |rho_h - rho_e|^2)^(1/2) over target cells, each sub-tet
        integrated with a Grundmann-Moeller rule of degree 2N+3."""
        from .quadrature import tet_rule
        pts, wts = tet_rule(2 * self.N + 3)
        phi = self.ref.eval_basis(pts)
        L = self.mesh["box"]
        tot = 0.0
        for c in self.targets:
            g = self.grids[c]
            uc = self.cell_state(u, c)[:, var]
            for k in range(len(g.conn)):
                x = g.X[k, 0] + pts @ g.J[k].T
                uh = phi @ uc[g.conn[k]]
                ue = exact_fn(x if self.bounded else np.mod(x, L))
                tot += g.detJ[k] * float(wts @ (uh - ue) ** 2)
        return math.sqrt(tot)
