"""Pins of the oracle's SU(N) basis and structure constants.

Each test checks the oracle against something fixed independently of it: the
orthonormality stated with the basis (Sec. II), the nonzero counts printed in
the paper (Sec. IV, step 2.2), textbook SU(2)/SU(3) tables, and group
identities (Casimir, Jacobi).
"""

import itertools
import math
import os

import numpy as np
import pytest

from oracle import basis

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_generators_orthonormal_hermitian_traceless(N):
    F = basis.generators(N)
    M = N * N - 1
    assert F.shape == (M, N, N)
    G = basis.gram(F)
    np.testing.assert_allclose(G, np.eye(M), atol=1e-14)
    # Gell-Mann scaling lambda = sqrt(2) F gives Tr(l_i l_j) = 2 delta_ij
    np.testing.assert_allclose(basis.gram(math.sqrt(2) * F), 2 * np.eye(M), atol=1e-14)
    for m in range(M):
        np.testing.assert_allclose(F[m], F[m].conj().T, atol=0)
        assert abs(np.trace(F[m])) < 1e-14
    # completeness: identity plus the M generators span all N x N matrices
    vecs = np.concatenate([np.eye(N).reshape(1, -1), F.reshape(M, -1)])
    assert np.linalg.matrix_rank(vecs) == N * N


def _read_counts():
    out = {}
    with open(os.path.join(GOLDEN, "nz_counts.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            n, a, b = (int(x) for x in line.split())
            out[n] = (a, b)
    return out


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 7, 8])
def test_nonzero_counts_match_paper(N):
    f, d = basis.structure_constants(N)
    fi, _ = basis.nonzero_triples(f)
    di, _ = basis.nonzero_triples(d)
    nzf, nzd = _read_counts()[N]
    assert len(fi) == nzf
    assert len(di) == nzd


@pytest.mark.parametrize("N", [3, 4, 5])
def test_f_antisymmetric_d_symmetric(N):
    f, d = basis.structure_constants(N)
    for perm in itertools.permutations(range(3)):
        sign = np.linalg.det(np.eye(3)[list(perm)])
        np.testing.assert_allclose(f.transpose(perm), sign * f, atol=1e-14)
        np.testing.assert_allclose(d.transpose(perm), d, atol=1e-14)


def test_su2_levi_civita():
    f, d = basis.structure_constants(2)
    # grouped order for N=2: S01 = sx/sqrt2, J01 = sy/sqrt2, D1 = sz/sqrt2
    eps = np.zeros((3, 3, 3))
    for (i, j, k), s in {(0, 1, 2): 1, (1, 2, 0): 1, (2, 0, 1): 1,
                         (0, 2, 1): -1, (2, 1, 0): -1, (1, 0, 2): -1}.items():
        eps[i, j, k] = s
    np.testing.assert_allclose(f, math.sqrt(2) * eps, atol=1e-14)
    np.testing.assert_allclose(d, 0, atol=1e-14)


def _read_su3():
    r3 = math.sqrt(3.0)
    rows = []
    with open(os.path.join(GOLDEN, "su3_gellmann.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            kind, a, b, c, val = line.split()
            rows.append((kind, int(a), int(b), int(c), eval(val, {"r3": r3})))
    return rows


def test_su3_matches_gell_mann_tables():
    f, d = basis.structure_constants(3)
    # Gell-Mann index (1..8) -> grouped index; N=3 order is
    # S01, S02, S12, J01, J02, J12, D1, D2
    pi = {1: 0, 2: 3, 3: 6, 4: 1, 5: 4, 6: 2, 7: 5, 8: 7}
    fg = np.zeros((9, 9, 9))
    dg = np.zeros((9, 9, 9))
    for kind, a, b, c, v in _read_su3():
        for perm in set(itertools.permutations((a, b, c))):
            if kind == "f":
                sign = np.linalg.det(np.eye(3)[[ (a, b, c).index(x) for x in perm ]])
                fg[perm] = sign * v
            else:
                dg[perm] = v
    for a in range(1, 9):
        for b in range(1, 9):
            for c in range(1, 9):
                assert abs(f[pi[a], pi[b], pi[c]] - math.sqrt(2) * fg[a, b, c]) < 1e-14
                assert abs(d[pi[a], pi[b], pi[c]] - math.sqrt(2) * dg[a, b, c]) < 1e-14


@pytest.mark.parametrize("N", [3, 4, 5, 6])
def test_casimir_identities(N):
    f, d = basis.structure_constants(N)
    M = N * N - 1
    np.testing.assert_allclose(np.einsum("mns,mnt->st", f, f), 2 * N * np.eye(M), atol=1e-12)
    np.testing.assert_allclose(np.einsum("mns,mnt->st", d, d),
                               2 * (N * N - 4) / N * np.eye(M), atol=1e-12)


@pytest.mark.parametrize("N", [3, 4])
def test_jacobi_identity(N):
    f, _ = basis.structure_constants(N)
    jac = (np.einsum("abe,ecd->abcd", f, f) + np.einsum("bce,ead->abcd", f, f)
           + np.einsum("cae,ebd->abcd", f, f))
    assert np.max(np.abs(jac)) < 1e-12


def test_nonzero_triples_sorted_and_planted_mistake_detected():
    f, d = basis.structure_constants(4)
    idx, vals = basis.nonzero_triples(f)
    keys = idx[:, 0] * 10**6 + idx[:, 1] * 10**3 + idx[:, 2]
    assert np.all(np.diff(keys) > 0)
    # a plausible indexing mistake (transposed last two indices) must break
    # the antisymmetry pin used above
    bad = f.transpose(0, 2, 1).copy()
    bad[0, 1, :] = f[0, 1, :]
    assert not np.allclose(bad.transpose(1, 0, 2), -bad, atol=1e-14)
