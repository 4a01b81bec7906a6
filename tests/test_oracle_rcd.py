"""Pins of the RCD oracle (Supplementary S4) against what the mathematics fixes
independently of its code: the circulant spectrum of D in closed form, exact
scaling of component-Fourier vectors by 1/(1 + dt k^2 lambda_j), the uncoupled
limit (scalar implicit diffusion), the homogeneous Lotka--Volterra equilibrium,
a hand-computed reaction for M = 3 and the M = 2 special case, brute-force
block geometry, threshold zero equal to dense, power-of-two invariance of the
masks, and Parseval for the measure."""
import numpy as np
import pytest

from oracle import rcd
from paper_2609_03922_amd import inputs

DD, DC, ALPHA, BETA, DT, DX = 0.5, 0.05, 1.0, 0.3, 0.01, 0.5


@pytest.mark.parametrize("M", [2, 3, 4, 8, 16])
def test_circulant_spectrum_closed_form(M):
    lam = np.sort(np.linalg.eigvalsh(rcd.diffusion_matrix(M, DD, DC)))
    if M == 2:
        want = np.array([DD + DC, DD + 3 * DC])
    else:
        want = np.sort(DD + 2 * DC - 2 * DC * np.cos(2 * np.pi * np.arange(M) / M))
    assert np.allclose(lam, want, rtol=0, atol=1e-14)
    assert rcd.diffusion_matrix(M, DD, DC)[0, 1] == -DC and np.count_nonzero(rcd.diffusion_matrix(M, DD, DC)[0]) == min(M, 3)


@pytest.mark.parametrize("M", [3, 5, 8])
def test_component_fourier_vector_is_scaled_exactly(M):
    # D is circulant: e_j(m) = exp(2 pi i j m / M) is an eigenvector with
    # lambda_j = DD + 2 DC (1 - cos(2 pi j / M)); with no reaction the update
    # divides it by 1 + dt k^2 lambda_j
    dims, block = (8, 8), (4, 4)
    N = 64
    k2 = rcd.k2(dims, DX)
    rng = np.random.default_rng(5)
    for j in range(M):
        e = np.exp(2j * np.pi * j * np.arange(M) / M)
        c = rng.normal(size=N) + 1j * rng.normal(size=N)
        q = e[:, None] * c[None, :]
        out = rcd.apply(q, np.zeros_like(q), dims, block, 0.0, DT, DX, DD, DC)["q"]
        lam = DD + 2 * DC * (1 - np.cos(2 * np.pi * j / M))
        want = q / (1.0 + DT * k2 * lam)[None, :]
        assert np.allclose(out, want, rtol=1e-13, atol=0)


def test_uncoupled_limit_is_scalar_implicit_diffusion():
    dims, block = (16, 16), (4, 4)
    M = 4
    q = np.stack([inputs.shaped_spectrum(11, m, dims, width=3.0).ravel() for m in range(M)])
    rh = np.stack([inputs.shaped_spectrum(12, m, dims, width=3.0).ravel() for m in range(M)])
    out = rcd.apply(q, rh, dims, block, 0.0, DT, DX, DD, 0.0)["q"]
    want = (q + DT * rh) / (1.0 + DT * DD * rcd.k2(dims, DX))[None, :]
    assert np.allclose(out, want, rtol=1e-13, atol=0)


def test_k2_closed_form():
    k2 = rcd.k2((4, 8), 0.5).reshape(4, 8)
    # index 3 of 4 is the frequency -1, index 4 of 8 is the Nyquist -4 (numpy's sign)
    w = 2 * np.pi
    assert np.isclose(k2[3, 0], (w * -1 / (4 * 0.5)) ** 2) and np.isclose(k2[0, 4], (w * -4 / (8 * 0.5)) ** 2)
    assert k2[0, 0] == 0.0


@pytest.mark.parametrize("M", [2, 3, 6])
def test_homogeneous_equilibrium_is_steady(M):
    us = rcd.equilibrium(M, ALPHA, BETA)
    # closed form: 1 / (1 + 2 (alpha + beta) + (M - 3) beta) for M >= 3, 1 / (1 + alpha + beta) for M = 2
    want = 1.0 / (1.0 + ALPHA + BETA) if M == 2 else 1.0 / (1.0 + 2 * (ALPHA + BETA) + (M - 3) * BETA)
    assert abs(us - want) <= 1e-15
    u = np.full((M, 4, 4), us)
    assert np.max(np.abs(rcd.reaction(u, ALPHA, BETA))) <= 1e-15
    dims = (4, 4, 4)
    q = np.stack([np.fft.fftn(np.full(dims, us)).ravel() for _ in range(M)])
    st = rcd.step(q, 5, dims, (2, 2, 2), 0.0, DT, DX, DD, DC, ALPHA, BETA)["state"]
    assert np.allclose(st, q, rtol=0, atol=1e-12 * abs(q[0, 0]))


def test_reaction_by_hand():
    # M = 3: every other component is a neighbour, alpha_ij = beta + alpha = 1.3
    u = np.array([1.0, 2.0, 3.0])
    R = rcd.reaction(u, ALPHA, BETA)
    assert np.allclose(R, [1 * (1 - 1 - 1.3 * 5), 2 * (1 - 2 - 1.3 * 4), 3 * (1 - 3 - 1.3 * 3)], rtol=1e-15)
    # M = 4: the opposite component interacts by beta only
    u = np.array([1.0, 2.0, 3.0, 4.0])
    R = rcd.reaction(u, ALPHA, BETA)
    assert np.isclose(R[0], 1 * (1 - 1 - 1.3 * 2 - 1.3 * 4 - 0.3 * 3), rtol=1e-15)
    # M = 2: the single other component, once
    R = rcd.reaction(np.array([0.5, 0.25]), ALPHA, BETA)
    assert np.allclose(R, [0.5 * (1 - 0.5 - 1.3 * 0.25), 0.25 * (1 - 0.25 - 1.3 * 0.5)], rtol=1e-15)


def test_block_geometry_and_single_mode():
    dims, block = (8, 16), (4, 4)
    bid = rcd.block_ids(dims, block)
    for z in range(8):
        for x in range(16):
            assert bid[z * 16 + x] == (z // 4) * 4 + x // 4
    M = 3
    q = np.zeros((M, 128), np.complex128)
    q[1, 5 * 16 + 9] = 3 - 4j       # block (1, 2) = 6, a = 25
    q[2, 5 * 16 + 9] = 1.0          # same mode, second component: a = 26
    q[0, 0] = 100.0                 # k = 0 is left out
    res = rcd.apply(q, np.zeros_like(q), dims, block, 0.5, DT, DX, DD, DC)
    assert res["G"] == 26.0 and res["a_b"][6] == 26.0 and res["a_b"].sum() == 26.0
    assert sorted(np.flatnonzero(res["mask"]).tolist()) == [0, 6]   # pinned k = 0 block
    res = rcd.apply(q, np.zeros_like(q), dims, block, 0.5, DT, DX, DD, DC, pin_k0=False)
    assert np.flatnonzero(res["mask"]).tolist() == [6]
    # frozen blocks keep their coefficients exactly
    assert np.array_equal(res["q"][:, bid != 6], q[:, bid != 6])


def test_threshold_zero_equals_dense_and_scaling():
    dims, block, M = (8, 8, 8), (4, 4, 4), 4
    u0 = inputs.perturbed_components(3, M, dims, rcd.equilibrium(M, ALPHA, BETA), 0.1)
    q = np.stack([np.fft.fftn(u0[m]).ravel() for m in range(M)])
    a = rcd.step(q, 4, dims, block, 0.0, DT, DX, DD, DC, ALPHA, BETA)["state"]
    b = rcd.step(q, 4, dims, block, 0.0, DT, DX, DD, DC, ALPHA, BETA, dense=True)["state"]
    assert np.array_equal(a, b)
    dims = (16, 16, 16)
    rh = np.stack([inputs.shaped_spectrum(13, m, dims, width=2.0).ravel() for m in range(M)])
    qs = np.stack([inputs.shaped_spectrum(14, m, dims, width=2.0).ravel() for m in range(M)])
    base = rcd.apply(qs, rh, dims, block, 0.1, DT, DX, DD, DC)
    assert 1 < base["count"] < 64
    for k in (-3, 5):
        s = rcd.apply(qs * 2.0 ** k, rh, dims, block, 0.1, DT, DX, DD, DC)
        assert np.array_equal(s["mask"], base["mask"]) and np.array_equal(s["a_b"], base["a_b"] * 4.0 ** k)


def test_measure_parseval():
    dims, M = (8, 8, 8), 3
    u = inputs.perturbed_components(4, M, dims, 0.2, 0.1)
    q = np.stack([np.fft.fftn(u[m]).ravel() for m in range(M)])
    a = rcd.measure(q)
    N = 512
    want = N * sum(float(np.sum((u[m] - u[m].mean()) ** 2)) for m in range(M))
    assert abs(a.sum() - want) <= 1e-11 * want


def test_eigen_form_identity():
    # S4.3: V (I + dt k^2 Lambda)^{-1} V^T equals the direct inverse
    M = 8
    D = rcd.diffusion_matrix(M, DD, DC)
    lam, V = np.linalg.eigh(D)
    for k2v in (0.0, 3.7, 150.0):
        Ai = np.linalg.inv(np.eye(M) + DT * k2v * D)
        Ae = V @ np.diag(1.0 / (1.0 + DT * k2v * lam)) @ V.T
        assert np.allclose(Ai, Ae, rtol=0, atol=1e-14)


@pytest.mark.parametrize("M", [2, 3, 7, 16, 64])
def test_solve_recovers_known_solutions(M):
    """The written-out elimination against systems whose solution is fixed in
    advance (b = A x for a chosen x), over the SPD matrices the update forms,
    a diagonal one (x = b / diag) and a matrix with wide coefficient range."""
    rng = np.random.default_rng(M)
    D = rcd.diffusion_matrix(M, DD, DC)
    s = np.array([0.0, 0.3, 17.0, 4e3])
    A = np.eye(M)[None] + s[:, None, None] * D[None]
    x = rng.normal(size=(s.size, M))
    b = np.einsum("nij,nj->ni", A, x)
    assert np.allclose(rcd.solve(A, b), x, rtol=0, atol=1e-12 * np.max(np.abs(x)))
    d = rng.uniform(0.5, 4.0, M)
    assert np.allclose(rcd.solve(np.diag(d)[None], d[None] * x[:1]), x[:1], rtol=1e-15, atol=0)
    Q = rng.normal(size=(M, M))
    S = Q @ Q.T + M * np.eye(M)
    assert np.allclose(S @ rcd.solve(S[None], b[:1])[0], b[0], rtol=0, atol=1e-11 * np.max(np.abs(b[0])))


def test_signed_index():
    assert list(rcd.signed_index(8)) == [0, 1, 2, 3, -4, -3, -2, -1]
    assert list(rcd.signed_index(1)) == [0]
