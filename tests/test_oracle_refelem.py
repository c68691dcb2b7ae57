"""Pins of the oracle's reference element against what the paper and the
mathematics fix (App. A closed forms, exact integrals, identities)."""
import itertools
from fractions import Fraction as Fr
from math import factorial, sqrt

import numpy as np
import pytest

from oracle.quadrature import tet_rule, tri_rule
from oracle.refelem import ref_element, ref_nodes, time_basis

RNG = np.random.default_rng(123)


def rand_pts(n):
    p = RNG.random((4 * n, 3))
    return p[p.sum(1) <= 1][:n]


def lam(p):
    r, s, t = p[:, 0], p[:, 1], p[:, 2]
    return 1 - r - s - t, r, s, t


@pytest.mark.parametrize("deg", [1, 3, 5, 7, 9])
def test_quadrature_exact_on_monomials(deg):
    pts, w = tet_rule(deg)
    for a, b, c in itertools.product(range(deg + 1), repeat=3):
        if a + b + c > deg:
            continue
        exact = factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)
        assert abs((w * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c).sum() - exact) < 1e-15
    tp, tw = tri_rule(deg)
    for a, b in itertools.product(range(deg + 1), repeat=2):
        if a + b <= deg:
            exact = factorial(a) * factorial(b) / factorial(a + b + 2)
            assert abs((tw * tp[:, 0] ** a * tp[:, 1] ** b).sum() - exact) < 1e-15


def test_p1_basis_and_mass_closed_form():
    """App. A P1: phi = barycentric coordinates; M^ = (1 + delta)/120 exactly."""
    R = ref_element(1)
    p = rand_pts(50)
    l1, l2, l3, l4 = lam(p)
    assert np.allclose(R.eval_basis(p), np.stack([l1, l2, l3, l4], 1), atol=1e-15)
    for m in range(4):
        for l in range(4):
            assert R.M[m][l] == Fr(1 + (m == l), 120)


def test_p2_basis_matches_appendix():
    """App. A P2 formulas, in the printed order."""
    R = ref_element(2)
    p = rand_pts(50)
    l1, l2, l3, l4 = lam(p)
    printed = [l1 * (2 * l1 - 1), l2 * (2 * l2 - 1), l3 * (2 * l3 - 1), l4 * (2 * l4 - 1),
               4 * l1 * l2, 4 * l2 * l3, 4 * l3 * l1, 4 * l1 * l4, 4 * l2 * l4, 4 * l3 * l4]
    assert np.allclose(R.eval_basis(p), np.stack(printed, 1), atol=1e-14)


def test_p3_printed_functions_are_the_basis_up_to_relabelling():
    """App. A P3: the 20 printed cubics are the Lagrange basis of the printed node
    lattice, but phi_7..phi_16 are listed against other nodes (e.g. the printed
    phi_7 is one at the listed x_10)."""
    R = ref_element(3)
    p = rand_pts(60)
    l1, l2, l3, l4 = lam(p)
    L = [l1, l2, l3, l4]
    printed = [0.5 * L[i] * (3 * L[i] - 1) * (3 * L[i] - 2) for i in range(4)]
    for i, j in [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]:
        printed += [4.5 * L[i] * L[j] * (3 * L[i] - 1), 4.5 * L[i] * L[j] * (3 * L[j] - 1)]
    printed += [27 * l1 * l2 * l3, 27 * l1 * l2 * l4, 27 * l1 * l3 * l4, 27 * l2 * l3 * l4]
    ours = R.eval_basis(p)
    match = []
    for f in printed:
        d = np.abs(ours - f[:, None]).max(0)
        assert d.min() < 1e-13
        match.append(int(d.argmin()))
    assert sorted(match) == list(range(20))
    assert match[6] == 9  # printed phi_7 is the Lagrange function of x_10


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_nodal_property_partition_of_unity_and_identities(N):
    R = ref_element(N)
    V = R.eval_basis(R.nodes_f)
    assert np.allclose(V, np.eye(R.np), atol=1e-13)
    p = rand_pts(40)
    assert np.allclose(R.eval_basis(p).sum(1), 1.0, atol=1e-13)
    assert sum(sum(r) for r in R.M) == Fr(1, 6)
    assert sum(sum(r) for r in R.Z) == Fr(1, 2)
    for d in range(3):
        for row in R.K[d]:
            assert sum(row) == 0  # sum_l d phi_l = 0
        for m in range(R.np):
            assert sum(R.D[d][m]) == 0


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_matrices_by_brute_force_quadrature(N):
    """M^, K^, D^ against Grundmann-Moeller quadrature and finite differences."""
    R = ref_element(N)
    pts, w = tet_rule(2 * N + 1)
    phi = R.eval_basis(pts)
    h = 1e-6
    dphi = []
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        dphi.append((R.eval_basis(pts + e) - R.eval_basis(pts - e)) / (2 * h))
    assert np.abs(np.einsum("q,qm,ql->ml", w, phi, phi) - R.M_f).max() < 1e-15
    for d in range(3):
        K = np.einsum("q,qm,ql->ml", w, phi, dphi[d])
        assert np.abs(K - R.K_f[d]).max() < 1e-8
        e = np.zeros(3)
        e[d] = h
        Dfd = (R.eval_basis(R.nodes_f + e) - R.eval_basis(R.nodes_f - e)) / (2 * h)
        assert np.abs(Dfd - R.D_f[d]).max() < 1e-6


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_stiffness_plus_transpose_is_boundary_mass(N):
    """K^_d + K^_d^T = int_T d_d(phi_m phi_l) = sum_faces n_d int_face phi_m phi_l,
    the face integrals done by quadrature on the four faces."""
    R = ref_element(N)
    tp, tw = tri_rule(2 * N + 1)
    faces = [  # (origin, edge1, edge2, outward normal * area scale)
        (np.zeros(3), np.array([1, 0, 0.]), np.array([0, 1, 0.]), np.array([0, 0, -1.]), 1.0),
        (np.zeros(3), np.array([1, 0, 0.]), np.array([0, 0, 1.]), np.array([0, -1, 0.]), 1.0),
        (np.zeros(3), np.array([0, 1, 0.]), np.array([0, 0, 1.]), np.array([-1, 0, 0.]), 1.0),
        (np.array([1, 0, 0.]), np.array([-1, 1, 0.]), np.array([-1, 0, 1.]), np.ones(3) / sqrt(3), sqrt(3)),
    ]
    B = np.zeros((3, R.np, R.np))
    for o, e1, e2, n, jac in faces:
        x = o + tp[:, :1] * e1 + tp[:, 1:] * e2
        ph = R.eval_basis(x)
        Mf = np.einsum("q,qm,ql->ml", tw * jac, ph, ph)
        for d in range(3):
            B[d] += n[d] * Mf
    for d in range(3):
        assert np.abs(R.K_f[d] + R.K_f[d].T - B[d]).max() < 1e-14


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_time_basis(N):
    tb = time_basis(N)
    assert abs(tb.w.sum() - 1.0) < 1e-15
    for k in range(2 * N + 2):
        assert abs((tb.w * tb.tau ** k).sum() - 1.0 / (k + 1)) < 1e-14
    assert np.allclose(tb.K_tau @ np.ones(N + 1), tb.psi0, atol=1e-13)
    # M_tau = int psi_a psi_b by an independent fine Gauss rule
    x, w = np.polynomial.legendre.leggauss(20)
    s, w = 0.5 * (x + 1), 0.5 * w
    P = np.array([[tb.psi(a, t) for a in range(N + 1)] for t in s])
    assert np.allclose(np.einsum("q,qa,qb->ab", w, P, P), tb.M_tau, atol=1e-14)


def test_time_operator_closed_form_n1():
    """N = 1: tau = 1/2 -+ sqrt(3)/6 and K_tau = [[1, (sqrt3-1)/2], [-(sqrt3+1)/2, 1]]."""
    tb = time_basis(1)
    r3 = sqrt(3.0)
    assert np.allclose(tb.tau, [0.5 - r3 / 6, 0.5 + r3 / 6], atol=1e-15)
    assert np.allclose(tb.K_tau, [[1.0, (r3 - 1) / 2], [-(r3 + 1) / 2, 1.0]], atol=1e-14)


def test_node_lists():
    assert [len(ref_nodes(N)) for N in (1, 2, 3, 4)] == [4, 10, 20, 35]
    assert ref_nodes(3)[9] == (0, Fr(1, 3), 0)
