"""Pins of the oracle's sector Hamiltonian (CPU only).

* Jordan-Wigner Fock-space construction (independent of the bit-string code)
  restricted to a sector equals the explicit sector matrix (Ns <= 5).
* H is symmetric with the hybridisation entries equal to +-V exactly.
* The explicit matrix built on full 2Ns-bit strings equals the Kronecker
  assembly H_d + H_up (x) 1 + 1 (x) H_dw (eq. Hdecomp, eq. Hbuild) entry for
  entry: so the spin-down sign does not depend on the spin-up string.
* Sampled rows of H.v (used for the Ns=16 sector) equal the explicit product.
* A planted mistake (a dropped string sign) is caught by the Jordan-Wigner pin.
"""
import numpy as np
import pytest

from oracle import fock, jw, kron
from paper_2105_06806_amd import inputs


TINY = [
    (dict(norb=1, nbath=3, U=2.0, seed=5), [(2, 2), (1, 3), (3, 2), (0, 4), (4, 4)]),
    (dict(norb=2, nbath=1, U=3.0, Jh=0.5, seed=6), [(2, 2), (1, 3), (2, 1), (3, 3)]),
    (dict(norb=1, nbath=4, U=1.3, seed=8), [(2, 3), (3, 2)]),
]


def _model(kw):
    kw = dict(kw)
    seed = kw.pop("seed")
    return inputs.make_model(kw.pop("norb"), kw.pop("nbath"), kw.pop("U"),
                             seed=seed, symmetric=False, **kw)


@pytest.mark.parametrize("kw,sectors", TINY)
def test_jordan_wigner_equals_explicit(kw, sectors):
    m = _model(kw)
    m["xmu"] = 0.37
    for (nu, nd) in sectors:
        A = jw.sector_block(m, nu, nd)
        B = fock.explicit_hamiltonian(m, nu, nd).toarray()
        assert np.allclose(A, B, rtol=0, atol=1e-13)


def test_planted_sign_error_is_caught():
    m = _model(TINY[0][0])
    A = jw.sector_block(m, 2, 2)
    orig = fock._parity_below
    try:
        fock._parity_below = lambda I, mm: np.ones(I.shape, dtype=np.int64)
        B = fock.explicit_hamiltonian(m, 2, 2).toarray()
    finally:
        fock._parity_below = orig
    assert not np.allclose(A, B, atol=1e-6)


@pytest.mark.parametrize("wl", ["ns8"])
def test_symmetric_and_pm_v(wl):
    m, [(nu, nd)] = inputs.workload(wl)
    H = fock.explicit_hamiltonian(m, nu, nd)
    assert (H != H.T).nnz == 0
    off = H - __import__("scipy.sparse", fromlist=["diags"]).diags(H.diagonal())
    vals = np.unique(np.abs(off.data[off.data != 0]))
    assert np.all(np.isin(vals, np.abs(m["vhyb"]).ravel()))


KRON_CASES = [
    (inputs.make_model(1, 7, 2.0, seed=1), (4, 4)),
    (inputs.make_model(1, 7, 2.0, seed=1), (5, 3)),
    (inputs.make_model(1, 9, 4.0, seed=2, symmetric=False), (4, 6)),
    (inputs.make_model(2, 3, 3.0, Jh=0.5, seed=3, symmetric=False), (4, 3)),
    (inputs.make_model(3, 2, 3.0, Jh=0.5, seed=4, symmetric=False), (4, 5)),
]


@pytest.mark.parametrize("m,sec", KRON_CASES)
def test_explicit_equals_kron_decomposition(m, sec):
    m = dict(m)
    m["xmu"] = 0.21
    H = fock.explicit_hamiltonian(m, *sec)
    K = kron.KronH(m, *sec)
    D = H.shape[0]
    assert K.dim == D
    # diagonal bitwise-equal up to summation order
    assert np.allclose(H.diagonal(), K.diagonal(), rtol=0, atol=1e-13)
    # off-diagonal: identical sparsity and values
    import scipy.sparse as sp
    Hup = sp.kron(sp.identity(K.Ddw), K.Hup, format="csr")
    Hdw = sp.kron(K.Hdw, sp.identity(K.Dup), format="csr")
    off = (H - sp.diags(H.diagonal())).tocsr()
    diff = off - (Hup + Hdw)
    diff.eliminate_zeros()
    assert diff.nnz == 0
    x = np.random.default_rng(0).standard_normal(D)
    assert np.allclose(K.matvec(x), H @ x, rtol=0, atol=1e-12)


@pytest.mark.parametrize("m,sec", KRON_CASES)
def test_sampled_rows(m, sec):
    H = fock.explicit_hamiltonian(m, *sec)
    x = np.random.default_rng(1).standard_normal(H.shape[0])
    rows = np.random.default_rng(2).choice(H.shape[0], size=min(300, H.shape[0]), replace=False)
    assert np.allclose(fock.hv_rows(m, *sec, x, rows), (H @ x)[rows], rtol=0, atol=1e-12)


def test_diagonal_terms_by_hand():
    # Norb=2, one bath level each: check the density-density energy of a few
    # hand-picked states against eq. Ham1 written out term by term.
    m = inputs.make_model(2, 1, 3.0, Jh=0.5, seed=9, symmetric=False)
    ns = 4
    e = fock.level_energies(m)
    U, Up, J = m["U"], m["Ust"], m["Jh"]
    # up: imp0 + imp1 occupied; dw: imp0 + bath(1) occupied
    Iup = 0b0011
    Idw = 0b1001
    I = np.array([Iup + (Idw << ns)], dtype=np.uint64)
    expect = (e[0] + e[1]) + (e[0] + e[3]) + U * 1 + Up * (1 * 0 + 1 * 1) + (Up - J) * 1
    assert np.isclose(fock.diagonal(m, I)[0], expect, rtol=0, atol=1e-14)
