"""Pins of the TVC oracle against brute force, closed forms and library
special cases (Sec. 3 definition).  CPU only."""
import itertools

import numpy as np
import pytest

from oracle import tvc as O
from paper_2501_03121_amd import synth

SHAPES = [(7,), (5, 3), (3, 1, 4), (2, 3, 5), (4, 1, 3, 2), (2, 3, 2, 2, 3), (2, 2, 1, 3, 2, 2)]


@pytest.mark.parametrize("dims", SHAPES)
def test_matches_brute_force(dims):
    A = synth.uniform(dims, 10)
    for k in range(len(dims)):
        x = synth.uniform(dims[k], 11 + k)
        np.testing.assert_allclose(O.tvc(A, x, k), O.tvc_loops(A, x, k), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dims", SHAPES)
def test_integer_inputs_are_exact(dims):
    A = synth.integers(dims, 20, -50, 50)
    for k in range(len(dims)):
        x = synth.integers(dims[k], 21 + k, -50, 50)
        assert np.array_equal(O.tvc(A, x, k), O.tvc_loops(A, x, k))


def test_one_hot_gives_slice():
    dims = (4, 5, 3, 2)
    A = synth.uniform(dims, 30)
    for k, n in enumerate(dims):
        for m in range(n):
            e = np.zeros(n)
            e[m] = 1.0
            assert np.array_equal(O.tvc(A, e, k), np.take(A, m, axis=k))


def test_ones_gives_mode_sum():
    dims = (3, 6, 4, 5)
    A = synth.integers(dims, 31, -9, 9)
    for k, n in enumerate(dims):
        assert np.array_equal(O.tvc(A, np.ones(n), k), A.sum(axis=k))


def test_contracting_all_modes_any_order():
    dims = (3, 4, 2, 5)
    A = synth.integers(dims, 40, -20, 20)
    xs = [synth.integers(n, 41 + i, -5, 5) for i, n in enumerate(dims)]
    ref = O.contract_all(A, xs, range(4))
    brute = sum(A[idx] * np.prod([xs[i][idx[i]] for i in range(4)])
                for idx in itertools.product(*[range(n) for n in dims]))
    assert ref == brute
    for order in itertools.permutations(range(4)):
        assert O.contract_all(A, xs, order) == ref


def test_order_two_is_gemv():
    A = synth.uniform((9, 7), 50)
    x1 = synth.uniform(7, 51)
    x0 = synth.uniform(9, 52)
    np.testing.assert_allclose(O.tvc(A, x1, 1), A @ x1, rtol=1e-14)
    np.testing.assert_allclose(O.tvc(A, x0, 0), x0 @ A, rtol=1e-14)


def test_moveaxis_equivalence_and_linearity():
    dims = (3, 4, 5, 2)
    A = synth.uniform(dims, 60)
    for k, n in enumerate(dims):
        x, z = synth.uniform(n, 61), synth.uniform(n, 62)
        np.testing.assert_allclose(O.tvc(A, x, k), O.tvc(np.moveaxis(A, k, -1), x, 3), rtol=1e-13)
        np.testing.assert_allclose(O.tvc(A, 2.0 * x - 3.0 * z, k),
                                   2.0 * O.tvc(A, x, k) - 3.0 * O.tvc(A, z, k), rtol=1e-12, atol=1e-12)


def test_alpha_beta_rules():
    A = synth.uniform((4, 3, 5), 70)
    x = synth.uniform(3, 71)
    y = synth.uniform((4, 5), 72)
    got = O.tvc(A, x, 1, alpha=-0.5, beta=2.0, y=y)
    np.testing.assert_allclose(got, -0.5 * O.tvc_loops(A, x, 1) + 2.0 * y, rtol=1e-13)
    nan = np.full((4, 5), np.nan)
    assert np.all(np.isfinite(O.tvc(A, x, 1, alpha=1.0, beta=0.0, y=nan)))


def test_sampled_outputs_match_full():
    dims = (6, 5, 7, 3)
    A = synth.uniform(dims, 80).astype(np.float32)
    for k, n in enumerate(dims):
        x = synth.uniform(n, 81)
        full = O.tvc(A, x, k)
        u, _, v = O.matricized_dims(dims, k)
        lr = np.stack([synth.rng(82).integers(0, u, 20), synth.rng(83).integers(0, v, 20)], axis=1)
        np.testing.assert_allclose(O.tvc_sample(A, x, k, lr), full.reshape(u, v)[lr[:, 0], lr[:, 1]],
                                   rtol=1e-14, atol=1e-14)


def test_matricized_dims_and_errors():
    assert O.matricized_dims((2, 3, 4), 0) == (1, 2, 12)
    assert O.matricized_dims((2, 3, 4), 1) == (2, 3, 4)
    assert O.matricized_dims((2, 3, 4), 2) == (6, 4, 1)
    with pytest.raises(ValueError):
        O.matricized_dims((2, 3), 2)
    with pytest.raises(ValueError):
        O.tvc(np.zeros((2, 3)), np.zeros(2), 1)


def test_rel_err():
    assert O.rel_err([1.0, 2.0], [1.0, 2.0]) == 0.0
    assert abs(O.rel_err([1.0, 0.0], [0.0, 0.0]) - 1.0) < 1e-15
