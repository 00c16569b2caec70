"""Pins of the HOPM oracle: exact rank-1 recovery, the matrix case against
the SVD, monotonicity, stationarity, Algorithm 1's contraction count and the
streamed-memory model Eq. (3).  CPU only."""
from pathlib import Path

import numpy as np
import pytest

from oracle import hopm as H
from oracle import tvc as O
from paper_2501_03121_amd import synth

GOLDEN = Path(__file__).parent / "golden"


@pytest.mark.parametrize("dims", [(6, 5, 4), (3, 4, 5, 2), (4, 3, 3, 2, 3)])
def test_exact_rank1_one_sweep(dims):
    a = synth.unit_vectors(dims, 1)
    T = np.ones(())
    for v in a:
        T = np.multiply.outer(T, v)
    x0 = synth.unit_vectors(dims, 3)
    r = H.hopm(7.5 * T, x0, sweeps=1)
    assert abs(r.lam - 7.5) < 1e-12
    for x, v in zip(r.xs, a):
        assert abs(abs(np.dot(x, v)) - 1.0) < 1e-12


def test_matrix_case_is_top_singular_triple():
    A = synth.normal((12, 9), 5)
    A += 6.0 * np.outer(synth.unit_vectors([12], 6)[0], synth.unit_vectors([9], 7)[0])
    r = H.hopm(A, synth.unit_vectors((12, 9), 8), tol=1e-13, max_sweeps=5000)
    U, S, Vt = np.linalg.svd(A)
    assert abs(r.lam - S[0]) < 1e-10 * S[0]
    assert abs(abs(np.dot(r.xs[0], U[:, 0])) - 1) < 1e-10
    assert abs(abs(np.dot(r.xs[1], Vt[0])) - 1) < 1e-10


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_norms_monotone_and_stationary(seed):
    dims = (9, 7, 8)
    A = synth.normal(dims, seed)
    r = H.hopm(A, synth.unit_vectors(dims, seed + 3), tol=1e-12, max_sweeps=3000)
    norms = np.array(r.norms)
    assert np.all(np.diff(norms) >= -1e-12 * norms[1:])
    for j in range(3):
        y = H.leave_one_out(A, r.xs, j)
        assert np.linalg.norm(y - r.lam * r.xs[j]) < 1e-9 * r.lam


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6])
def test_algorithm1_matches_canonical_and_counts(d):
    dims = tuple([3, 4, 2, 3, 2, 3][:d])
    A = synth.normal(dims, 11)
    x0 = synth.unit_vectors(dims, 12)
    c = H.hopm(A, x0, sweeps=4)
    a = H.dhopm3(A, x0, sweeps=4)
    for u, v in zip(c.xs, a.xs):
        np.testing.assert_allclose(u, v, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(c.norms, a.norms, rtol=1e-12)
    assert c.tvcs == 4 * d * (d - 1)
    assert a.tvcs == 4 * (d - 1) * (d + 2) // 2 == 4 * H.tvcs_per_sweep_dhopm3(d)
    # the paper states the saving as (d-1)(d-2)/2 contractions per sweep
    assert (c.tvcs - a.tvcs) // 4 == (d - 1) * (d - 2) // 2


@pytest.mark.parametrize("n,d", [(5, 2), (4, 3), (3, 4), (3, 5), (2, 6)])
def test_eq3_streamed_memory(n, d):
    dims = (n,) * d
    r = H.hopm(synth.normal(dims, 21), synth.unit_vectors(dims, 22), sweeps=1)
    assert r.touched == d * H.m_seq(n, d)
    a = H.dhopm3(synth.normal(dims, 21), synth.unit_vectors(dims, 22), sweeps=1)
    assert a.touched == H.dhopm3_touched(n, d)


def test_streamed_ratio_fig2():
    # The paper reads about 1.5x saving for the order-3 and roughly fivefold for
    # the order-10 tensor of Table 1 (Fig. 2(b), one process).
    r3 = H.streamed_ratio(979, 3)
    r10 = H.streamed_ratio(8, 10)
    assert 1.45 < r3 < 1.55
    assert 4.5 < r10 < 5.5


def test_table1_sizes():
    rows = [ln.split() for ln in (GOLDEN / "table1_hypersquare.txt").read_text().splitlines()
            if ln and not ln.startswith("#")]
    gbs = []
    for d, n, gb in rows:
        if d == "avg":
            assert abs(np.mean(gbs) - float(gb)) < 0.005
            continue
        size = int(n) ** int(d) * 8 / 1e9
        assert round(size, 2) == float(gb)
        gbs.append(float(gb))


def test_planted_tiny_config_recovers():
    dims = (64, 64, 64)
    A, a = synth.planted_rank1(dims, 5.0, 0.01, 100)
    r = H.hopm(A, synth.unit_vectors(dims, 103), sweeps=20)
    assert abs(r.lam - 5.0) < 0.05
    for x, v in zip(r.xs, a):
        assert abs(np.dot(x, v)) > 0.9999


def test_degenerate_zero_tensor():
    with pytest.raises(H.DegenerateError):
        H.hopm(np.zeros((3, 4, 2)), synth.unit_vectors((3, 4, 2), 0), sweeps=1)


def test_lambda_is_full_contraction():
    dims = (5, 4, 6)
    A = synth.normal(dims, 31)
    r = H.hopm(A, synth.unit_vectors(dims, 32), sweeps=3)
    assert abs(O.contract_all(A, r.xs, range(3)) - r.lam) < 1e-12 * r.lam


def _loo_brute(A, xs, j):
    # every multi-index of A, one product per element (tiny tensors only)
    import itertools
    y = np.zeros(A.shape[j])
    for idx in itertools.product(*[range(n) for n in A.shape]):
        p = float(A[idx])
        for i, x in enumerate(xs):
            if i != j:
                p *= float(x[idx[i]])
        y[idx[j]] += p
    return y


@pytest.mark.parametrize("dims", [(7, 5), (3, 4, 5), (2, 3, 4, 3), (3, 2, 2, 3, 2)])
@pytest.mark.parametrize("block,workers", [(1 << 26, 1), (7, 1), (1, 1), (7, 3)])
def test_kron_leave_one_out_brute_force(dims, block, workers):
    A = synth.normal(dims, 21)
    xs = [synth.uniform(n, 22 + i) for i, n in enumerate(dims)]
    for j in range(len(dims)):
        ref = _loo_brute(A, xs, j)
        got = H.leave_one_out_kron(A, xs, j, block_elems=block, workers=workers)
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
        if workers > 1:
            # threads change nothing: the block results are added in order
            np.testing.assert_array_equal(got, H.leave_one_out_kron(A, xs, j, block_elems=block))
        np.testing.assert_allclose(H.leave_one_out(A, xs, j), ref, rtol=1e-12, atol=1e-12)


def test_kron_leave_one_out_rank1_closed_form():
    dims = (4, 6, 5, 3)
    a = synth.unit_vectors(dims, 31)
    T = np.ones(())
    for v in a:
        T = np.multiply.outer(T, v)
    xs = [synth.uniform(n, 32 + i) for i, n in enumerate(dims)]
    for j in range(4):
        c = 2.5 * np.prod([np.dot(a[i], xs[i]) for i in range(4) if i != j])
        np.testing.assert_allclose(H.leave_one_out_kron(2.5 * T, xs, j, block_elems=5), c * a[j],
                                   rtol=1e-12, atol=1e-14)


def test_kron_order_of_kronecker_vector():
    # last vector fastest: (a (x) b)[i * len(b) + k] = a[i] b[k]
    a, b = np.array([1.0, 2.0]), np.array([3.0, 5.0, 7.0])
    np.testing.assert_array_equal(H.kron([a, b]), [3, 5, 7, 6, 10, 14])
    np.testing.assert_array_equal(H.kron([]), [1.0])


@pytest.mark.parametrize("dims", [(9, 7, 8), (3, 4, 2, 3, 5, 2, 3), (2, 3, 2, 3, 2, 2, 3, 2, 2)])
def test_kron_form_hopm_equals_chain(dims):
    A = synth.normal(dims, 41)
    x0 = synth.unit_vectors(dims, 42)
    c = H.hopm(A, x0, sweeps=5)
    k = H.hopm(A, x0, sweeps=5, form="kron")
    np.testing.assert_allclose(k.norms, c.norms, rtol=1e-12)
    np.testing.assert_allclose(k.deltas, c.deltas, rtol=1e-9, atol=1e-14)
    for u, v in zip(k.xs, c.xs):
        np.testing.assert_allclose(u, v, rtol=1e-11, atol=1e-12)
    # a float32 input is upcast exactly: same as passing its float64 copy
    A32 = A.astype(np.float32)
    k32 = H.hopm(A32, x0, sweeps=2, form="kron")
    k64 = H.hopm(A32.astype(np.float64), x0, sweeps=2, form="kron")
    np.testing.assert_array_equal(k32.norms, k64.norms)


@pytest.mark.parametrize("k", [1, 2, 5])
def test_jacobi_matrix_case_is_two_power_iterations(k):
    # d = 2: x_0 after 2k Jacobi sweeps is (A A^T)^k x_0 normalised (up to sign)
    A = synth.normal((11, 8), 51)
    x0 = synth.unit_vectors((11, 8), 52)
    r = H.jacobi_hopm(A, x0, sweeps=2 * k)
    v0 = np.linalg.matrix_power(A @ A.T, k) @ x0[0]
    v1 = np.linalg.matrix_power(A.T @ A, k) @ x0[1]
    assert abs(abs(np.dot(r.xs[0], v0 / np.linalg.norm(v0))) - 1) < 1e-12
    assert abs(abs(np.dot(r.xs[1], v1 / np.linalg.norm(v1))) - 1) < 1e-12


@pytest.mark.parametrize("dims", [(6, 5, 4), (3, 4, 5, 2), (4, 3, 3, 2, 3), (5, 7)])
def test_jacobi_exact_rank1(dims):
    a = synth.unit_vectors(dims, 61)
    T = np.ones(())
    for v in a:
        T = np.multiply.outer(T, v)
    r = H.jacobi_hopm(7.5 * T, synth.unit_vectors(dims, 62), sweeps=3)
    for x, v in zip(r.xs, a):
        assert abs(abs(np.dot(x, v)) - 1.0) < 1e-12
    # every vector is +-a_j after one sweep; the sign choice keeps it still
    assert r.deltas[1] < 1e-12 and r.deltas[2] < 1e-12
    assert abs(r.lams[1] - 7.5) < 1e-12


@pytest.mark.parametrize("dims", [(5, 4, 6), (3, 4, 2, 3)])
def test_jacobi_first_sweep_uses_previous_vectors(dims):
    A = synth.normal(dims, 71)
    x0 = synth.unit_vectors(dims, 72)
    r = H.jacobi_hopm(A, x0, sweeps=1)
    for j in range(len(dims)):
        y = _loo_brute(A, x0, j)
        y = y / np.linalg.norm(y)
        if np.dot(y, x0[j]) < 0:
            y = -y
        np.testing.assert_allclose(r.xs[j], y, rtol=1e-12, atol=1e-13)
    # the Gauss-Seidel sweep differs after j = 0
    g = H.hopm(A, x0, sweeps=1)
    np.testing.assert_allclose(g.xs[0], r.xs[0] * np.sign(np.dot(g.xs[0], r.xs[0])), rtol=1e-12)
    assert np.linalg.norm(np.abs(g.xs[1]) - np.abs(r.xs[1])) > 1e-6


@pytest.mark.parametrize("dims", [(12, 10, 9), (6, 5, 7, 4)])
def test_jacobi_reaches_the_gauss_seidel_fixed_point(dims):
    A, a = synth.planted_rank1(dims, 6.0, 0.05, 81, noise_kind="normal")
    x0 = synth.unit_vectors(dims, 82)
    gs = H.hopm(A, x0, tol=1e-13, max_sweeps=5000)
    ja = H.jacobi_hopm(A, x0, tol=1e-13, max_sweeps=5000)
    assert ja.deltas[-1] < 1e-13
    assert abs(ja.lam - gs.lam) < 1e-11 * gs.lam
    for u, v in zip(ja.xs, gs.xs):
        assert abs(abs(np.dot(u, v)) - 1) < 1e-11
    # kron form: same iterates
    jk = H.jacobi_hopm(A, x0, sweeps=6, form="kron")
    jc = H.jacobi_hopm(A, x0, sweeps=6)
    np.testing.assert_allclose(jk.norms, jc.norms, rtol=1e-12)
