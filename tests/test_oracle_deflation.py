"""Pins of the oracle's deflated estimator (Sec. Deflation) against closed
forms and exact identities, independent of the GPU library:

* free-field eigenvalues m2 + sum_mu 4 sin^2(pi n_mu / D_mu) (Fourier modes),
* Tr(P A^{-1} Q) for a complete low shell of free-field modes in closed form,
* with every site its own colour the deflated estimate equals Tr(P A^{-1})
  exactly for any noise and ANY basis V (the split is an identity: checked
  with eigenvectors and with a random basis, against the Fourier closed form
  and a dense inverse),
* the exact variance of the deflated estimator (eq. (2) reading for complex
  noise applied to P A^{-1} (I - Q)) is below the undeflated one and matches
  Monte Carlo.
"""
import itertools

import numpy as np
import pytest

import oracle
import workloads

D4 = (4, 4, 4, 4)


def _free_spectrum(dims, m2):
    ev = []
    for n in itertools.product(*[range(d) for d in dims]):
        ev.append(m2 + sum(4 * np.sin(np.pi * k / d) ** 2 for k, d in zip(n, dims)))
    return np.sort(np.array(ev))


@pytest.mark.parametrize("nc", [1, 3])
def test_free_field_eigenvalues(nc):
    m2 = 0.5
    w, V = oracle.lowest_eigenpairs(D4, nc, m2, None, 40)
    exact = np.repeat(_free_spectrum(D4, m2), nc)[:40]
    assert np.max(np.abs(w - exact)) < 1e-12
    Vm = V.reshape(40, -1)
    assert np.max(np.abs(Vm.conj() @ Vm.T - np.eye(40))) < 1e-12


def test_deflated_part_closed_form_free_field():
    """The lowest shell of the 4^4 free field: the constant mode (m2) and the
    eight modes with one momentum component +-1 (m2 + 2).  For p = 1 the
    modes with n_0 = +-1 contribute cos(pi/2) = 0, so
    Tr(P A^{-1} Q) = 1/m2 + 6/(m2 + 2)."""
    m2 = 0.5
    _, V = oracle.lowest_eigenpairs(D4, 1, m2, None, 9)
    col = np.zeros(256, dtype=np.int32)
    r = oracle.trace_deflated(D4, 1, m2, None, 1, col, 1, 3, 0, 2, oracle.Z2_COMPLEX, False, V)
    assert abs(r["T_defl"] - (1 / m2 + 6 / (m2 + 2))) < 1e-12
    # p = 0: every mode counts
    r0 = oracle.trace_deflated(D4, 1, m2, None, 0, col, 1, 3, 0, 1, oracle.Z2_COMPLEX, False, V)
    assert abs(r0["T_defl"] - (1 / m2 + 8 / (m2 + 2))) < 1e-12


@pytest.mark.parametrize("basis", ["eigen", "random"])
def test_all_distinct_colours_exact_free_field(basis):
    m2, p = 0.5, 1
    exact, _ = workloads.free_field_trace(D4, m2, p)
    if basis == "eigen":
        _, V = oracle.lowest_eigenpairs(D4, 1, m2, None, 9)
    else:
        rng = np.random.default_rng(5)
        V = rng.standard_normal((5, 256, 1)) + 1j * rng.standard_normal((5, 256, 1))
    col = np.arange(256, dtype=np.int32)
    r = oracle.trace_deflated(D4, 1, m2, None, p, col, 256, 7, 0, 1, oracle.Z2_COMPLEX, False, V)
    assert abs(r["T"] - exact) < 1e-11 * abs(exact)


@pytest.mark.parametrize("p", [0, 2])
def test_all_distinct_colours_exact_gauge(p):
    U = workloads.random_links(D4, 0.3, 1)
    A = oracle.dense(D4, 3, 0.1, U)
    rows = oracle.shift(D4, np.arange(768).reshape(256, 3), p).reshape(768)
    exact = np.sum(np.linalg.inv(A)[rows, np.arange(768)])
    _, V = oracle.lowest_eigenpairs(D4, 3, 0.1, U, 12)
    col = np.arange(256, dtype=np.int32)
    r = oracle.trace_deflated(D4, 3, 0.1, U, p, col, 256, 11, 0, 1, oracle.Z2_COMPLEX, True, V)
    assert abs(r["T"] - exact) < 1e-10 * abs(exact)


def test_deflation_reduces_variance():
    """Hutchinson (one colour) on the 4^4 free field, m2 = 0.05: exact
    per-sample variance sum_{i != j} |B_ij|^2 (complex noise, E z^2 = 0) of
    B = P A^{-1} and of B = P A^{-1} (I - Q), and Monte Carlo for the latter."""
    m2, p, nvec = 0.05, 1, 9
    A = oracle.dense(D4, 1, m2, None)
    _, V = oracle.lowest_eigenpairs(D4, 1, m2, None, nvec)
    Vm = V.reshape(nvec, -1).T
    Pm = np.zeros((256, 256))
    rows = oracle.shift(D4, np.arange(256).reshape(256, 1), p).reshape(256)
    Pm[np.arange(256), rows] = 1
    Ainv = np.linalg.inv(A)
    B0 = Pm @ Ainv
    B1 = Pm @ Ainv @ (np.eye(256) - Vm @ Vm.conj().T)

    def var(B):
        return np.sum(np.abs(B) ** 2) - np.sum(np.abs(np.diag(B)) ** 2)
    v0, v1 = var(B0), var(B1)
    assert v1 < 0.2 * v0
    col = np.zeros(256, dtype=np.int32)
    r = oracle.trace_deflated(D4, 1, m2, None, p, col, 1, 2, 0, 400, oracle.Z2_COMPLEX, False, V)
    mc = np.var(r["per_sample"], ddof=1)
    assert abs(mc / v1 - 1) < 0.25
    assert abs(r["T"] - np.trace(B0)) < 5 * np.sqrt(v1 / 400)
