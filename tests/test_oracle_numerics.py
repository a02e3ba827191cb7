"""Pins for the oracle's noise, operator, CG, probed trace and adjoint gradient.

The oracle is checked against dense linear algebra (numpy), the free-field
Fourier closed form, exact identities of the probed estimator (Sec. 2.1-2.2,
eq. (2) in its corrected reading) and central finite differences.
"""
import numpy as np
import pytest

import oracle
import workloads

D4 = (4, 4, 4, 4)
D2 = (2, 2, 2, 2)


@pytest.fixture(scope="module")
def gauge4():
    U = workloads.random_links(D4, 0.3, 1)
    A = oracle.dense(D4, 3, 0.1, U)
    return U, A


def _perm_matrix(dims, p):
    """(P v)(x) = v(x + p e0) as a dense matrix over (site, colour) pairs."""
    N = int(np.prod(dims))
    P = np.zeros((N, N))
    for i in range(N):
        x = np.array(np.unravel_index(i, dims))
        x[0] = (x[0] + p) % dims[0]
        P[i, np.ravel_multi_index(tuple(x), dims)] = 1
    return P


# ------------------------------------------------------------------ noise


def test_mix64_is_a_bijection_on_a_sample_and_fixes_zero():
    assert oracle.mix64(0) == 0
    vals = {oracle.mix64(i) for i in range(1, 5000)}
    assert len(vals) == 4999


def test_mix64_is_the_splitmix64_output_function():
    """The noise hash is SplitMix64's output function (Steele, Lea and
    Flood, OOPSLA 2014): the generator seeded with 0 adds the golden-ratio
    increment 0x9E3779B97F4A7C15 to its state and outputs mix64(state); its
    published first outputs are reproduced exactly."""
    gamma = 0x9E3779B97F4A7C15
    published = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC,
                 0x1B39896A51A8749B]
    for i, want in enumerate(published, start=1):
        assert oracle.mix64((gamma * i) % 2 ** 64) == want


@pytest.mark.parametrize("kind", [oracle.REAL_Z2, oracle.Z2_COMPLEX, oracle.Z4])
def test_noise_statistics(kind):
    """Rademacher / Z4 noise (Sec. 2): mean 0, E|z|^2 = 1 after the
    normalisation, E z^2 = 0 for complex noise, values in the right set,
    adjacent counters uncorrelated."""
    col = np.zeros(4096, dtype=np.int32)
    z = np.concatenate([oracle.probe((16, 16, 4, 4), 3, col, 7, s, 0, 0, False, kind).ravel()
                        for s in range(4)])
    n = z.size
    norm = oracle.noise_norm(kind)
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert np.allclose(norm * np.abs(z) ** 2, 1.0)
    if kind == oracle.REAL_Z2:
        assert set(np.unique(z.real)) == {-1.0, 1.0} and np.all(z.imag == 0)
    elif kind == oracle.Z2_COMPLEX:
        assert set(np.unique(z.real)) == {-1.0, 1.0} == set(np.unique(z.imag))
        assert abs((z ** 2).mean()) < 10 / np.sqrt(n)
    else:
        assert np.all((np.abs(z.real) + np.abs(z.imag)) == 1)
        assert abs((z ** 2).mean()) < 10 / np.sqrt(n)
        for v in (1, 1j, -1, -1j):  # each value with probability 1/4
            assert abs(np.mean(z == v) - 0.25) < 5 * np.sqrt(0.1875 / n)
    assert abs(np.mean(np.conj(z[:-1]) * z[1:])) < 10 / np.sqrt(n)


def test_probe_masks_and_dilution():
    """eq. (3)-(4): the probe is z0 on the sites of one colour (and, diluted,
    one colour component); the probes of a sample sum to z0."""
    col, n, _ = oracle.coloring(D4, 1, 2, oracle.NATURAL)
    P = oracle.probes(D4, 3, col, n, 5, 2, 1, oracle.Z4, True)
    assert P.shape == (n * 3, 256, 3)
    z0 = P.sum(axis=0)
    assert np.all(np.abs(z0) == 1)
    for j in range(P.shape[0]):
        c, a = j // 3, j % 3
        mask = np.zeros((256, 3), dtype=bool)
        mask[col == c, a] = True
        assert np.array_equal(P[j][mask], z0[mask]) and np.all(P[j][~mask] == 0)


# ------------------------------------------------------------------ operator


def test_operator_free_field_spectrum():
    """U = 1: eigenvalues m2 + sum_mu 4 sin^2(k_mu/2) (Fourier closed form)."""
    A = oracle.dense(D4, 1, 0.5, None)
    ks = np.meshgrid(*[2 * np.pi * np.arange(4) / 4] * 4, indexing="ij")
    lam = 0.5 + sum(4 * np.sin(k / 2) ** 2 for k in ks)
    assert np.allclose(np.sort(np.linalg.eigvalsh(A)), np.sort(lam.ravel()), atol=1e-12)


def test_operator_hermitian_and_bounded(gauge4):
    U, A = gauge4
    assert np.allclose(A, A.conj().T, atol=1e-14)
    w = np.linalg.eigvalsh(A)
    assert w.min() >= 0.1 - 1e-12 and w.max() <= 0.1 + 16 + 1e-12


def test_operator_gauge_covariance(gauge4):
    """U_mu(x) -> g(x) U_mu(x) g(x+mu)^H gives A -> G A G^H (this fixes the
    link orientation and the neighbour each link multiplies)."""
    U, A = gauge4
    N = 256
    g = workloads.random_links(D4, 1.0, 99)[0]
    Ug = np.empty_like(U)
    for mu in range(4):
        for i in range(N):
            x = np.array(np.unravel_index(i, D4))
            x[mu] = (x[mu] + 1) % 4
            j = np.ravel_multi_index(tuple(x), D4)
            Ug[mu, i] = g[i] @ U[mu, i] @ g[j].conj().T
    G = np.zeros((3 * N, 3 * N), dtype=complex)
    for i in range(N):
        G[3 * i:3 * i + 3, 3 * i:3 * i + 3] = g[i]
    Ag = oracle.dense(D4, 3, 0.1, Ug)
    assert np.allclose(Ag, G @ A @ G.conj().T, atol=1e-12)


def test_operator_identity_links_is_free_field():
    U = np.zeros((4, 256, 3, 3), dtype=complex)
    U[:] = np.eye(3)
    v = np.random.default_rng(0).standard_normal((256, 3)) + 0j
    w = oracle.apply(D4, 3, 0.5, U, v)
    for a in range(3):
        assert np.allclose(w[:, a], oracle.apply(D4, 1, 0.5, None, v[:, a:a + 1])[:, 0])


# ------------------------------------------------------------------ CG


def test_cg_matches_dense_solve(gauge4):
    U, A = gauge4
    b = np.random.default_rng(1).standard_normal(768) + 1j * np.random.default_rng(2).standard_normal(768)
    x, it, rel = oracle.cg(D4, 3, 0.1, U, b.reshape(256, 3), tol=1e-13)
    assert it > 0 and rel < 1e-12
    assert np.allclose(x.ravel(), np.linalg.solve(A, b), rtol=0, atol=1e-10 * np.abs(b).max())


def test_cg_free_field_terminates_in_nine_iterations():
    """4^4 free field: 9 distinct eigenvalues m2 + {0, 2, ..., 16}, so CG
    terminates in at most 9 steps in exact arithmetic."""
    col, n, _ = oracle.coloring(D4, 1, 2, oracle.NATURAL)
    z = oracle.probe(D4, 1, col, 0, 0, 0, 0, False, oracle.REAL_Z2)
    _, it, rel = oracle.cg(D4, 1, 0.5, None, z, tol=1e-12)
    assert 0 < it <= 9 and rel < 1e-11


def test_cg_failure_modes():
    z = oracle.probe(D4, 1, np.zeros(256, np.int32), 0, 0, 0, 0, False, oracle.REAL_Z2)
    _, it, _ = oracle.cg(D4, 1, 0.5, None, z, tol=1e-12, maxit=2)
    assert it == -2
    _, it, _ = oracle.cg(D4, 1, -9.0, None, z, tol=1e-12)  # A negative definite
    assert it == -1


# ------------------------------------------------------------------ trace


def test_free_field_trace_exact_with_all_distinct_colours():
    """With every site its own colour, probing recovers Tr(P A^{-1}) exactly
    for any noise (Sec. 2.1): compare with the Fourier closed form (4^4, m2=0.5,
    p=1: 6.73722476756959)."""
    exact, dexact = workloads.free_field_trace(D4, 0.5, 1)
    assert abs(exact - 6.73722476756959) < 1e-12
    col = np.arange(256, dtype=np.int32)
    r = oracle.trace(D4, 1, 0.5, None, 1, col, 256, 3, 0, 1, oracle.REAL_Z2, False, tol=1e-13)
    assert abs(r["T"] - exact) < 1e-11 * abs(exact)
    T, g, _, _ = oracle.trace_grad(D4, 1, 0.5, None, 1, col, 256, 3, 0, 1, oracle.REAL_Z2, False,
                                   tol=1e-13)
    assert abs(g - dexact) < 1e-10 * abs(dexact) and abs(T - exact) < 1e-11 * abs(exact)


@pytest.mark.parametrize("p", [0, 1, 2, -1])
def test_gauge_trace_exact_with_all_distinct_colours(gauge4, p):
    """Dense inverse: Tr(P A^{-1}) = sum_x A^{-1}[x + p e0, x] (Sec. 3)."""
    U, A = gauge4
    B = np.kron(_perm_matrix(D4, p % 4), np.eye(3)) @ np.linalg.inv(A)
    col = np.arange(256, dtype=np.int32)
    r = oracle.trace(D4, 3, 0.1, U, p, col, 256, 11, 0, 1, oracle.Z2_COMPLEX, True, tol=1e-13)
    assert abs(r["T"] - np.trace(B)) < 1e-10 * abs(np.trace(B))


def test_negative_displacement_is_conjugate(gauge4):
    U, A = gauge4
    col = np.arange(256, dtype=np.int32)
    a = oracle.trace(D4, 3, 0.1, U, 1, col, 256, 0, 0, 1, oracle.Z4, True, tol=1e-13)["T"]
    b = oracle.trace(D4, 3, 0.1, U, -1, col, 256, 0, 0, 1, oracle.Z4, True, tol=1e-13)["T"]
    assert abs(a - np.conj(b)) < 1e-10 * abs(a)


@pytest.mark.parametrize("kind,dilute", [(oracle.Z2_COMPLEX, True), (oracle.Z4, False),
                                         (oracle.REAL_Z2, True)])
def test_probed_sample_identity(gauge4, kind, dilute):
    """For a fixed noise sample (eqs. (1), (3), (4)):
    T_s - Tr(B) = norm * sum_{i != j, same class} conj(z0_i) B_ij z0_j, with
    B = P A^{-1}, class = colour (and colour component when diluted)."""
    U, A = gauge4
    p = 1
    B = np.kron(_perm_matrix(D4, p), np.eye(3)) @ np.linalg.inv(A)
    col, n, _ = oracle.coloring(D4, p, 2, oracle.NATURAL)
    r = oracle.trace(D4, 3, 0.1, U, p, col, n, 21, 0, 3, kind, dilute, tol=1e-13)
    norm = oracle.noise_norm(kind)
    cls = np.repeat(col, 3) * 3 + (np.tile(np.arange(3), 256) if dilute else 0)
    same = cls[:, None] == cls[None, :]
    np.fill_diagonal(same, False)
    for s in range(3):
        z0 = oracle.probes(D4, 3, col, n, 21, s, 1, kind, dilute).sum(axis=0).ravel()
        want = np.trace(B) + norm * (np.conj(z0) @ (B * same) @ z0)
        assert abs(r["per_sample"][s] - want) < 1e-10 * abs(want)
    assert abs(r["T"] - r["per_sample"].mean()) < 1e-12 * abs(r["T"])


def test_variance_identity_monte_carlo():
    """Corrected eq. (2) for the probed estimator on the 4^4 free field
    (p=1, distance-2 colouring, 8 colours): real noise gives
    Var(T_s) = sum_{i<j same colour} (B_ij + B_ji)^2; the per-sample variance
    is 0.674371 probed against 13.9477 unprobed.  Checked by Monte Carlo with
    the oracle's own noise."""
    A = oracle.dense(D4, 1, 0.5, None)
    B = _perm_matrix(D4, 1) @ np.linalg.inv(A).real
    col, n, _ = oracle.coloring(D4, 1, 2, oracle.NATURAL)
    assert n == 8

    def var_of(colors):
        same = colors[:, None] == colors[None, :]
        S = (B + B.T) ** 2 * np.triu(same, 1)
        return S.sum()

    v_probed, v_plain = var_of(col), var_of(np.zeros(256, np.int64))
    assert abs(v_probed - 0.674371) < 1e-6 and abs(v_plain - 13.9477) < 1e-4
    ts = []
    for s in range(4000):
        z0 = oracle.probes(D4, 1, col, n, 3, s, 1, oracle.REAL_Z2, False).sum(axis=0).ravel().real
        ts.append(sum(z0[col == c] @ B[np.ix_(col == c, col == c)] @ z0[col == c] for c in range(n)))
    ts = np.array(ts)
    assert abs(ts.mean() - np.trace(B)) < 5 * np.sqrt(v_probed / len(ts))
    assert abs(ts.var(ddof=1) / v_probed - 1) < 5 * np.sqrt(2 / len(ts))


def test_variance_identity_complex_noise(gauge4):
    """Complex noise with E z^2 = 0: Var(T_s) = sum_{i != j same class} |B_ij|^2."""
    U, A = gauge4
    B = np.kron(_perm_matrix(D4, 1), np.eye(3)) @ np.linalg.inv(A)
    col, n, _ = oracle.coloring(D4, 1, 2, oracle.NATURAL)
    cls = np.repeat(col, 3) * 3 + np.tile(np.arange(3), 256)
    same = cls[:, None] == cls[None, :]
    np.fill_diagonal(same, False)
    v = np.sum(np.abs(B[same]) ** 2)
    ts = []
    for s in range(1500):
        z0 = oracle.probes(D4, 3, col, n, 9, s, 1, oracle.Z2_COMPLEX, True).sum(axis=0).ravel()
        ts.append(0.5 * (np.conj(z0) @ (B * (same | np.eye(768, dtype=bool))) @ z0))
    ts = np.array(ts)
    assert abs(np.mean(np.abs(ts - np.trace(B)) ** 2) / v - 1) < 5 * np.sqrt(2 / len(ts))


# ------------------------------------------------------------------ gradient


def _su3_direction(rng, N):
    G = rng.standard_normal((4, N, 3, 3)) + 1j * rng.standard_normal((4, N, 3, 3))
    X = 0.5 * (G + np.conj(np.swapaxes(G, -1, -2)))
    X -= np.trace(X, axis1=-2, axis2=-1)[..., None, None] / 3 * np.eye(3)
    return X


def _expm_herm(X, h):
    w, Q = np.linalg.eigh(X)
    return (Q * np.exp(1j * h * w)[..., None, :]) @ np.conj(np.swapaxes(Q, -1, -2))


@pytest.mark.parametrize("dims,p", [(D2, 1), (D4, 1)])
def test_gradient_central_differences(dims, p):
    """dT/dm2 and dT/dU against central differences (h = 1e-4) along
    U(h) = exp(i h X) U with random su(3) directions X, fixed probes:
    dT/dh = sum [dT/dU . (i X U) + dT/dUbar . conj(i X U)]."""
    N = int(np.prod(dims))
    U = workloads.random_links(dims, 0.5, 3)
    m2 = 0.2
    col, n, _ = oracle.coloring(dims, p, 2, oracle.NATURAL)
    args = (p, col, n, 17, 0, 1, oracle.Z2_COMPLEX, True)
    T, g, dU, dUb = oracle.trace_grad(dims, 3, m2, U, *args, tol=1e-14)
    T0 = oracle.trace(dims, 3, m2, U, *args, tol=1e-14)["T"]
    assert abs(T - T0) < 1e-12 * abs(T0)
    h = 1e-4
    Tp = oracle.trace(dims, 3, m2 + h, U, *args, tol=1e-14)["T"]
    Tm = oracle.trace(dims, 3, m2 - h, U, *args, tol=1e-14)["T"]
    assert abs((Tp - Tm) / (2 * h) - g) < 1e-6 * abs(g)
    rng = np.random.default_rng(5)
    ndir = 16 if N <= 16 else 4
    for _ in range(ndir):
        X = _su3_direction(rng, N)
        Up, Um = _expm_herm(X, h) @ U, _expm_herm(X, -h) @ U
        fd = (oracle.trace(dims, 3, m2, Up, *args, tol=1e-14)["T"]
              - oracle.trace(dims, 3, m2, Um, *args, tol=1e-14)["T"]) / (2 * h)
        dUdh = 1j * X @ U
        an = np.sum(dU * dUdh) + np.sum(dUb * np.conj(dUdh))
        assert abs(fd - an) < 1e-6 * max(abs(an), 1e-3), (fd, an)


def test_contractions_equal_the_trace_per_rhs_terms():
    """The numpy contraction of the oracle's own solutions equals the per-
    right-hand-side terms t_j of its C trace (two restatements of Sec. 3's
    z^H P x), for p = 0, 1 and -1 on a 3-colour gauge lattice, and for p = 0
    its sum is the dense Hutchinson sum of the probes."""
    dims, nc, m2 = (4, 2, 3, 2), 3, 0.3
    U = workloads.random_links(dims, 0.4, 5, nc)
    col, n, _ = oracle.coloring(dims, 1, 1, oracle.NATURAL)
    V = oracle.probes(dims, nc, col, n, 9, 0, 1, oracle.Z2_COMPLEX, True)
    X, its, rel = oracle.cg_many(dims, nc, m2, U, V, tol=1e-13)
    assert (its > 0).all()
    for p in (0, 1, -1):
        t = oracle.contractions(dims, nc, V, X, p)
        ref = oracle.trace(dims, nc, m2, U, p % dims[0], col, n, 9, 0, 1, oracle.Z2_COMPLEX, True,
                           tol=1e-13)["tj"]
        assert np.abs(t - ref).max() < 1e-12 * np.abs(ref).max(), p
    Ainv = np.linalg.inv(oracle.dense(dims, nc, m2, U))
    t0 = oracle.contractions(dims, nc, V, X, 0)
    want = sum(np.vdot(v.ravel(), Ainv @ v.ravel()) for v in V)
    assert abs(t0.sum() - want) < 1e-10 * abs(want)
