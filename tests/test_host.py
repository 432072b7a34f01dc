"""Host-side checks of the library (no GPU): symbol table, MPO construction against the
oracle's FCI Hamiltonian and Slater-Condon rules, error paths."""
import os
import re

import numpy as np
import pytest

import synth
from oracle import fci, slater
from paper_1902_08489_amd import tdmps as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return T.load()


def test_library_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "tdmps.h")).read()
    declared = sorted(set(re.findall(r"\b(tdmps_[A-Za-z0-9_]+)\s*\(", hdr)))
    assert len(declared) >= 30
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(T.symbols()) == declared


@pytest.mark.parametrize("window", [None, "-1", "0", "1", "6"])
@pytest.mark.parametrize("L", [2, 3, 4, 5, 6])
def test_mpo_equals_fci_on_fock_space(lib, L, window, monkeypatch):
    """The MPO contracted to a 4^L x 4^L matrix is the Hamiltonian of Eq. (hamil), for every
    routing of the pair channels (plain rule, adjacent-operator rule at the centre cut, within
    one cut of it, everywhere, and the default window)."""
    if window is not None:
        monkeypatch.setenv("TDMPS_MPO_ROUTING_WINDOW", window)
    h, eri, _ = synth.integrals(L, seed=40 + L)
    M = T.MPO.from_integrals(None, h, eri, 0.31)
    H = fci.hamiltonian(fci.Space.full(L), h, eri, 0.31).toarray()
    assert np.abs(M.to_dense() - H).max() < 1e-12


def test_mpo_bond_dimension_formula(lib, monkeypatch):
    """Channel count at the chain centre under the plain rule: I, H, 4L single-operator
    channels, and the pair channels of the left half: 2 + 4L + 2 C(L,2) + L^2 = 2L^2 + 3L + 2.
    The default routing adds the pairs next to an operator site near the centre, and leaves
    the chain ends alone."""
    for L in (6, 8, 12, 16, 24):
        h, eri, _ = synth.integrals(L)
        monkeypatch.setenv("TDMPS_MPO_ROUTING_WINDOW", "-1")
        d = T.MPO.from_integrals(None, h, eri).bond_dims()
        assert d[L // 2] == 2 * L * L + 3 * L + 2
        assert d[0] == 1 and d[L] == 1
        monkeypatch.delenv("TDMPS_MPO_ROUTING_WINDOW")
        r = T.MPO.from_integrals(None, h, eri).bond_dims()
        assert r[L // 2] > d[L // 2]
        w = L // 6
        assert np.array_equal(r[: L // 2 - w], d[: L // 2 - w]) and np.array_equal(r[L // 2 + w + 1:], d[L // 2 + w + 1:])


@pytest.mark.parametrize("L", [24, 30])
def test_mpo_matches_slater_condon_at_full_size(lib, L):
    """<D'|H|D> through the MPO equals the Slater-Condon rules for coinciding, singly and
    doubly differing determinants at the benchmark sizes."""
    h, eri, _ = synth.integrals(L)
    M = T.MPO.from_integrals(None, h, eri, 0.5)
    sc = slater.SlaterCondon(h, eri, 0.5)
    rng = np.random.default_rng(L)
    occ = synth.ionized_determinant(L, L)
    m0 = slater.occ_to_mask(occ)
    cases = [(m0, m0)]
    occs = [j for j in range(2 * L) if (m0 >> j) & 1]
    virt = [j for j in range(2 * L) if not (m0 >> j) & 1]
    for _ in range(12):
        i = int(rng.choice(occs))
        a = int(rng.choice([v for v in virt if (v & 1) == (i & 1)]))
        cases.append((m0 ^ (1 << i) ^ (1 << a), m0))
        i2 = int(rng.choice([o for o in occs if o != i]))
        a2 = int(rng.choice([v for v in virt if v != a and (v & 1) == (i2 & 1)]))
        cases.append((m0 ^ (1 << i) ^ (1 << a) ^ (1 << i2) ^ (1 << a2), m0))
    for bra, ket in cases:
        ob = np.array([((bra >> (2 * p)) & 1) | (((bra >> (2 * p + 1)) & 1) << 1) for p in range(L)], np.uint8)
        ok = np.array([((ket >> (2 * p)) & 1) | (((ket >> (2 * p + 1)) & 1) << 1) for p in range(L)], np.uint8)
        want = sc.element(bra, ket)
        assert abs(M.det_element(ob, ok) - want) < 1e-11 * max(1.0, abs(want))


def test_set_one_body_and_dipole_operator(lib):
    """Replacing h in place gives the MPO of the new Hamiltonian; the one-body MPO is
    sum_pq t_pq E_pq."""
    L = 4
    h, eri, _ = synth.integrals(L)
    mu = synth.dipole_matrix(L)
    M = T.MPO.from_integrals(None, h, eri, 0.0)
    M.set_one_body(h + 0.3 * mu)
    space = fci.Space.full(L)
    assert np.abs(M.to_dense() - fci.hamiltonian(space, h + 0.3 * mu, eri).toarray()).max() < 1e-12
    D = T.MPO.one_body(None, mu)
    assert np.abs(D.to_dense() - fci.one_body_operator(space, mu).toarray()).max() < 1e-12
    assert D.bond_dims().max() <= 2 + 4 * L


def test_error_paths(lib):
    L = 3
    h, eri, _ = synth.integrals(L)
    bad = h.copy()
    bad[0, 1] = np.nan
    with pytest.raises(T.TdmpsError) as e:
        T.MPO.from_integrals(None, bad, eri)
    assert e.value.code == -5
    M = T.MPO.from_integrals(None, h, eri)
    with pytest.raises(T.TdmpsError) as e:
        M.det_element(np.array([0, 4, 1], np.uint8), np.array([0, 1, 1], np.uint8))
    assert e.value.code == -1
    with pytest.raises(T.TdmpsError):
        T.MPO.from_integrals(None, np.zeros((1, 1)), np.zeros((1,) * 4))


def test_fiedler_order_host(lib):
    """Orbital order of the H2O section through the C ABI (host code only): the oracle's
    permutation on scrambled integrals, a scrambled chain restored, NaN rejected."""
    from oracle import ordering
    rng = np.random.default_rng(12)
    for L in (5, 9, 16):
        h, eri, _ = synth.integrals(L, seed=70 + L)
        P = rng.permutation(L)
        hs, es = ordering.permute(h, eri, P)
        assert list(T.fiedler_order(hs, es)) == list(ordering.fiedler_order(hs, es))
        chain = np.diag(np.linspace(-1, 1, L)) - 0.5 * (np.eye(L, k=1) + np.eye(L, k=-1))
        back = P[T.fiedler_order(chain[np.ix_(P, P)])]
        assert list(back) in (list(range(L)), list(range(L))[::-1])
    bad = np.eye(4)
    bad[0, 2] = bad[2, 0] = np.inf
    with pytest.raises(T.TdmpsError):
        T.fiedler_order(bad)
