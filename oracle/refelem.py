"""Reference tetrahedron T^ = {r, s, t >= 0, r + s + t <= 1} (App. A).

Nodes follow the listing of App. A for N = 1, 2, 3.  The basis is defined by
the nodal property phi_j(x_m) = delta_jm on those nodes (Sec. 4.1).  For N = 3
the printed formulas pair phi_7..phi_16 with other nodes than the printed
list (e.g. the printed phi_7 equals one at (0, 1/3, 0), the listed x_10); the
node list is taken as the definition and each basis function is the Lagrange
function of its node, which makes the printed set of 20 polynomials and this
set equal up to relabelling.

All reference integrals are exact rationals from the monomial formula
    int_T^ r^a s^b t^c = a! b! c! / (a + b + c + 3)!
    int_K^ r^a s^b     = a! b! / (a + b + 2)!        (reference triangle)
and are converted to float64 only at the end.
"""
from __future__ import annotations

from fractions import Fraction as Fr
from functools import lru_cache
from math import factorial

import numpy as np

__all__ = ["ref_nodes", "RefElement", "ref_element", "TimeBasis", "time_basis"]


def ref_nodes(N: int) -> list[tuple[Fr, Fr, Fr]]:
    """Interpolation nodes of the P_N element in App. A order."""
    o, h, t3, tt3 = Fr(0), Fr(1, 2), Fr(1, 3), Fr(2, 3)
    verts = [(o, o, o), (Fr(1), o, o), (o, Fr(1), o), (o, o, Fr(1))]
    if N == 1:
        return verts
    if N == 2:
        return verts + [(h, o, o), (h, h, o), (o, h, o), (o, o, h), (h, o, h), (o, h, h)]
    if N == 3:
        return verts + [
            (t3, o, o), (tt3, o, o),
            (tt3, t3, o), (t3, tt3, o),
            (o, tt3, o), (o, t3, o),
            (o, o, t3), (o, o, tt3),
            (t3, o, tt3), (tt3, o, t3),
            (o, t3, tt3), (o, tt3, t3),
            (t3, t3, o), (t3, o, t3), (o, t3, t3), (t3, t3, t3),
        ]
    if N == 4:
        # App. A.4 defines the 35 nodes as the lattice r, s, t in {0, 1/4, 1/2,
        # 3/4, 1}, r + s + t <= 1, without listing them (its edge and face
        # counts, 12 and 18, are swapped: 6 edges carry 3 nodes each, 4 faces
        # 3 each, one node is interior).  Order taken: the vertices as above,
        # then edge, face and interior nodes, each group lexicographic in
        # (r, s, t).
        lat = [(Fr(i, 4), Fr(j, 4), Fr(k, 4)) for i in range(5) for j in range(5 - i) for k in range(5 - i - j)]

        def entity(p):
            lam = (1 - sum(p),) + p
            return sum(1 for x in lam if x != 0) - 1

        rest = sorted((p for p in lat if p not in verts), key=lambda p: (entity(p), p))
        return verts + rest
    raise ValueError("N must be 1, 2, 3 or 4")


def _monomials(N: int) -> list[tuple[int, int, int]]:
    return [(a, b, c) for a in range(N + 1) for b in range(N + 1 - a) for c in range(N + 1 - a - b)]


def _solve_exact(A: list[list[Fr]], B: list[list[Fr]]) -> list[list[Fr]]:
    """Gauss-Jordan elimination over the rationals: returns A^{-1} B."""
    n = len(A)
    M = [row[:] + brow[:] for row, brow in zip(A, B)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        inv = 1 / M[col][col]
        M[col] = [x * inv for x in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    return [row[n:] for row in M]


def _tet_int(a: int, b: int, c: int) -> Fr:
    return Fr(factorial(a) * factorial(b) * factorial(c), factorial(a + b + c + 3))


def _tri_int(a: int, b: int) -> Fr:
    return Fr(factorial(a) * factorial(b), factorial(a + b + 2))


class RefElement:
    """Exact P_N reference data on T^.

    Attributes (Fraction lists and float64 arrays of the same name + '_f'):
        nodes      [np][3]       reference node coordinates
        coef       [nmono][np]   monomial coefficients of each basis function
        M          [np][np]      M^_{ml} = int phi_m phi_l
        K          [3][np][np]   K^_d,{ml} = int phi_m d_d phi_l   (eqn.Kspace, spatial part)
        V          [3][np][np]   V^_d,{ml} = int d_d phi_m phi_l = K^_d^T
        D          [3][np][np]   D^_d,{ml} = d_d phi_l (x_m)   (collocated derivative)
        face_nodes [nf]          reference nodes on the face t = 0, in node order
        Z          [nf][nf]      face mass on the reference triangle (area 1/2)
    """

    def __init__(self, N: int):
        self.N = N
        self.nodes = ref_nodes(N)
        self.np = len(self.nodes)
        assert self.np == (N + 1) * (N + 2) * (N + 3) // 6
        mono = _monomials(N)
        self.mono = mono
        V = [[Fr(x[0]) ** a * Fr(x[1]) ** b * Fr(x[2]) ** c for (a, b, c) in mono] for x in self.nodes]
        # basis_j = sum_p coef[p][j] mono_p with V coef = I
        ident = [[Fr(int(i == j)) for j in range(self.np)] for i in range(self.np)]
        self.coef = _solve_exact(V, ident)
        npn = self.np
        nm = len(mono)
        # products of monomials
        def mono_int(p, q, dq=None):
            a = mono[p][0] + mono[q][0]
            b = mono[p][1] + mono[q][1]
            c = mono[p][2] + mono[q][2]
            return _tet_int(a, b, c)

        Mmono = [[mono_int(p, q) for q in range(nm)] for p in range(nm)]
        # derivative of monomial q in direction d: coefficient and exponent
        def dmono(q, d):
            e = list(mono[q])
            k = e[d]
            if k == 0:
                return Fr(0), None
            e[d] -= 1
            return Fr(k), tuple(e)

        Kmono = [[[Fr(0)] * nm for _ in range(nm)] for _ in range(3)]
        for d in range(3):
            for p in range(nm):
                for q in range(nm):
                    f, e = dmono(q, d)
                    if e is None:
                        continue
                    Kmono[d][p][q] = f * _tet_int(mono[p][0] + e[0], mono[p][1] + e[1], mono[p][2] + e[2])
        C = self.coef

        def congruence(Mm):
            # (C^T Mm C)_{ml} = sum_pq C[p][m] Mm[p][q] C[q][l]
            tmp = [[sum(Mm[p][q] * C[q][l] for q in range(nm)) for l in range(npn)] for p in range(nm)]
            return [[sum(C[p][m] * tmp[p][l] for p in range(nm)) for l in range(npn)] for m in range(npn)]

        self.M = congruence(Mmono)
        self.K = [congruence(Kmono[d]) for d in range(3)]
        self.V = [[[self.K[d][l][m] for l in range(npn)] for m in range(npn)] for d in range(3)]
        # collocated derivatives D_d[m][l] = d_d phi_l(x_m)
        self.D = []
        for d in range(3):
            Dd = [[Fr(0)] * npn for _ in range(npn)]
            for m, x in enumerate(self.nodes):
                for l in range(npn):
                    val = Fr(0)
                    for q in range(nm):
                        f, e = dmono(q, d)
                        if e is None or C[q][l] == 0:
                            continue
                        val += C[q][l] * f * Fr(x[0]) ** e[0] * Fr(x[1]) ** e[1] * Fr(x[2]) ** e[2]
                    Dd[m][l] = val
            self.D.append(Dd)
        # face t = 0 : its nodes and the restricted basis
        self.face_nodes = [m for m, x in enumerate(self.nodes) if x[2] == 0]
        fn = self.face_nodes
        nf = len(fn)
        assert nf == (N + 1) * (N + 2) // 2
        Z = [[Fr(0)] * nf for _ in range(nf)]
        for i, m in enumerate(fn):
            for j, l in enumerate(fn):
                val = Fr(0)
                for p in range(nm):
                    if mono[p][2] != 0 or C[p][m] == 0:
                        continue
                    for q in range(nm):
                        if mono[q][2] != 0 or C[q][l] == 0:
                            continue
                        val += C[p][m] * C[q][l] * _tri_int(mono[p][0] + mono[q][0], mono[p][1] + mono[q][1])
                Z[i][j] = val
        self.Z = Z
        f64 = lambda A: np.array([[float(x) for x in row] for row in A])
        self.nodes_f = np.array([[float(c) for c in x] for x in self.nodes])
        self.M_f = f64(self.M)
        self.K_f = np.stack([f64(k) for k in self.K])
        self.V_f = np.stack([f64(v) for v in self.V])
        self.D_f = np.stack([f64(dd) for dd in self.D])
        self.Z_f = f64(self.Z)
        self.face_nodes_a = np.array(fn, dtype=np.int64)

    def eval_basis(self, pts: np.ndarray) -> np.ndarray:
        """phi_j at reference points pts [n, 3] -> [n, np] (float64)."""
        pts = np.asarray(pts, dtype=np.float64)
        P = np.stack([pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c for (a, b, c) in self.mono], axis=1)
        return P @ np.array([[float(x) for x in row] for row in self.coef])

    def barycentric_weights(self) -> np.ndarray:
        """Integer barycentric weights N*(lambda1..lambda4) of each node, with
        lambda1 = 1 - r - s - t, lambda2 = r, lambda3 = s, lambda4 = t (App. A)."""
        out = []
        for x in self.nodes:
            l2, l3, l4 = (c * self.N for c in x)
            l1 = self.N - l2 - l3 - l4
            out.append([int(l1), int(l2), int(l3), int(l4)])
        return np.array(out, dtype=np.int64)


@lru_cache(maxsize=None)
def ref_element(N: int) -> RefElement:
    return RefElement(N)


class TimeBasis:
    """Lagrange basis psi_a through the N+1 Gauss-Legendre points of [0, 1]
    (Sec. 4.3: space-time basis is the tensor product of the spatial basis and
    this one; the number of time nodes is not stated, N+1 is taken).

        tau, w   nodes and weights on [0, 1] (numpy leggauss, mapped)
        M_tau    int psi_a psi_b           = diag(w)  (exact: degree 2N <= 2N+1)
        K_tau    psi_a(1) psi_b(1) - int psi_a' psi_b   (upwind time operator of K_1)
        psi0     psi_a(0)   (the F_0 matrix is psi(0) (x) M^)
        psi1     psi_a(1)
    """

    def __init__(self, N: int):
        nt = N + 1
        x, w = np.polynomial.legendre.leggauss(nt)
        self.tau = 0.5 * (x + 1.0)
        self.w = 0.5 * w
        self.nt = nt
        tau = self.tau

        def psi(a, s):
            v = 1.0
            for b in range(nt):
                if b != a:
                    v *= (s - tau[b]) / (tau[a] - tau[b])
            return v

        def dpsi(a, s):
            tot = 0.0
            for c in range(nt):
                if c == a:
                    continue
                v = 1.0 / (tau[a] - tau[c])
                for b in range(nt):
                    if b != a and b != c:
                        v *= (s - tau[b]) / (tau[a] - tau[b])
                tot += v
            return tot

        self.psi0 = np.array([psi(a, 0.0) for a in range(nt)])
        self.psi1 = np.array([psi(a, 1.0) for a in range(nt)])
        # int_0^1 psi_a' psi_b = sum_c w_c psi_a'(tau_c) psi_b(tau_c) = w_b psi_a'(tau_b)
        self.K_tau = np.array([[self.psi1[a] * self.psi1[b] - self.w[b] * dpsi(a, tau[b]) for b in range(nt)]
                               for a in range(nt)])
        self.M_tau = np.diag(self.w)
        self.K_tau_inv = np.linalg.inv(self.K_tau)
        self.psi = psi
        self.dpsi = dpsi


@lru_cache(maxsize=None)
def time_basis(N: int) -> TimeBasis:
    return TimeBasis(N)
