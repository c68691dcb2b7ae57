"""The oracle's reference element against the nodes and basis functions the
paper prints in its appendix on P1-P3 (fixture tests/golden/appendix_basis.txt,
exact fractions).  The printed P3 list numbers some cubics against other nodes
than the printed node list does, so for P3 the match is up to relabelling."""
import os
import re
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle.refelem import ref_element, ref_nodes

HERE = os.path.dirname(os.path.abspath(__file__))


def _load():
    nodes, phis = {}, {}
    with open(os.path.join(HERE, "golden", "appendix_basis.txt")) as f:
        for ln in f:
            tok = ln.split()
            if not tok or tok[0].startswith("#"):
                continue
            N, i = int(tok[1]), int(tok[2])
            if tok[0] == "node":
                nodes.setdefault(N, {})[i] = tuple(Fr(v) for v in tok[3:6])
            else:
                phis.setdefault(N, {})[i] = (Fr(tok[3]), tok[4:])
    return ({N: [d[i] for i in sorted(d)] for N, d in nodes.items()},
            {N: [d[i] for i in sorted(d)] for N, d in phis.items()})


NODES, PHIS = _load()


def _bary(p):
    r, s, t = p
    return (1 - r - s - t, r, s, t)


def _eval(phi, lam):
    """Printed formula at barycentric coordinates lam (Fractions or arrays)."""
    coef, factors = phi
    out = coef
    for fa in factors:
        m = re.fullmatch(r"(\d+)l(\d)-(\d+)", fa)
        if m:
            out = out * (int(m.group(1)) * lam[int(m.group(2)) - 1] - int(m.group(3)))
        else:
            out = out * lam[int(re.fullmatch(r"l(\d)", fa).group(1)) - 1]
    return out


@pytest.mark.parametrize("N", [1, 2, 3])
def test_printed_nodes_are_the_oracle_nodes(N):
    assert len(NODES[N]) == len(PHIS[N]) == (N + 1) * (N + 2) * (N + 3) // 6
    assert sorted(NODES[N]) == sorted(ref_nodes(N))
    if N < 3:  # P1 and P2 are printed in the oracle's order
        assert NODES[N] == ref_nodes(N)


@pytest.mark.parametrize("N", [1, 2, 3])
def test_printed_functions_are_lagrange_on_printed_nodes(N):
    """Exact arithmetic: the matrix phi_i(x_j) is a permutation, the identity
    for P1 and P2."""
    V = np.array([[_eval(phi, _bary(x)) for x in NODES[N]] for phi in PHIS[N]], dtype=object)
    assert all(v in (0, 1) for v in V.ravel())
    P = V.astype(int)
    assert (P.sum(0) == 1).all() and (P.sum(1) == 1).all()
    if N < 3:
        assert (P == np.eye(len(P), dtype=int)).all()
    else:
        assert not (P == np.eye(len(P), dtype=int)).all()  # the relabelling noted above


@pytest.mark.parametrize("N", [1, 2, 3])
def test_oracle_basis_equals_printed_functions(N):
    """At random points each printed function equals the oracle's basis
    function of the node where it is one."""
    R = ref_element(N)
    rng = np.random.default_rng(11)
    p = rng.random((400, 3))
    p = p[p.sum(1) <= 1][:60]
    lam = (1 - p.sum(1), p[:, 0], p[:, 1], p[:, 2])
    ours = R.eval_basis(p)
    order = ref_nodes(N)
    for phi in PHIS[N]:
        at = [x for x in NODES[N] if _eval(phi, _bary(x)) == 1]
        assert len(at) == 1
        col = order.index(at[0])
        f = np.asarray(_eval(phi, [np.asarray(v, dtype=float) for v in lam]), dtype=float)
        assert np.abs(ours[:, col] - f).max() < 1e-13


def test_p4_nodes_are_the_appendix_lattice():
    """App. A.4 defines the 35 quartic nodes as all (r, s, t) with r, s, t in
    {0, 1/4, 1/2, 3/4, 1} and r + s + t <= 1, with the four vertices, one
    interior node at (1/4, 1/4, 1/4), and the rest on edges and faces (the
    printed counts, 12 on edges and 18 on faces, are swapped: a tetrahedron's
    6 edges carry 3 lattice nodes each and its 4 faces 3 each)."""
    q = [Fr(i, 4) for i in range(5)]
    lattice = sorted((r, s, t) for r in q for s in q for t in q if r + s + t <= 1)
    nodes = ref_nodes(4)
    assert len(nodes) == 35 and sorted(nodes) == lattice
    assert nodes[:4] == [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    entity = [sum(1 for x in _bary(p) if x != 0) - 1 for p in nodes]
    assert [entity.count(d) for d in range(4)] == [4, 18, 12, 1]
    assert nodes[entity.index(3)] == (Fr(1, 4), Fr(1, 4), Fr(1, 4))
    assert entity == sorted(entity)  # vertices, edges, faces, interior
